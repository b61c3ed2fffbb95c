#!/usr/bin/env python3
"""Benchmark: batched RK4 integration of 4096 independent antennal-lobe-shaped
Hodgkin-Huxley networks on one MI355X, against the plain one-network-per-launch
form and the FP64 CPU oracle.

One bench step = one launch of the batched persistent kernel (a graph launch)
advancing every instance by --chunk RK4 steps, with spike detection and a V
trace every 100 steps.  Inputs are resident in HBM before timing starts.

Prints one JSON line (see the keys at the end of main()).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "neuron-RK4-steps/s batched vs plain at stated error; adjoint steps/s"
HBM_PEAK_GBS = 8000.0
DT = 0.01
REC_STRIDE = 100
SPIKE_CAP = 64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stratified(sizes, k):
    order = np.argsort(sizes, kind="stable")
    return [int(b) for b in order[np.linspace(0, len(sizes) - 1, k).astype(int)]]


def _counter_rows(path, kernel_substr, counter, by_name=False):
    import csv
    out = []
    for r in csv.DictReader(open(path)):
        if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter:
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            out.append((r["Kernel_Name"], dur, float(r["Counter_Value"])) if by_name
                       else (dur, float(r["Counter_Value"])))
    return out


def _per_launch(path, kernel_substr, counter):
    """Counter value of one launch summed over its dispatches.  A batch
    launches one kernel per launch group (a group is a kernel name and grid
    size; two groups may run the same kernel); the groups of the run's last
    launch are the dispatches from the last one back to the first repeated
    group (the launches are sequential; under counter collection so are a
    launch's own dispatches).  For each of those groups, the mean over its
    dispatches within 75 % of its longest (the timed launches, not the
    tuner's shorter runs of the same group), summed over the groups; groups
    the tuner alone ran are not in the last launch.  Returns (value,
    dispatches counted per group)."""
    import csv
    disp = []
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        if kernel_substr not in name or r["Counter_Name"] != counter:
            continue
        grid = r.get("Grid_Size") or r.get("Grid_Size_X")
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        disp.append((t0, (name, grid), t1 - t0, float(r["Counter_Value"])))
    if not disp:
        return 0.0, 0
    disp.sort(key=lambda d: d[0])
    final = set()
    for _, key, _, _ in reversed(disp):
        if key in final:
            break
        final.add(key)
    total, n = 0.0, 0
    for key in final:
        rows = [(d, v) for _, k, d, v in disp if k == key]
        longest = max(d for d, _ in rows)
        vals = [v for d, v in rows if d > 0.75 * longest]
        total += float(np.mean(vals))
        n = max(n, len(vals))
    return total, n


# the sources each profiled kernel is compiled from: a counter figure is used
# only while they are unchanged
KERNEL_SOURCES = {
    # the batched launch: the LDS-resident kernel and the lane-group kernel
    "rk4_wg_kernel": ("rk4_wg.hip", "wg_common.h", "hh_device.h", "kernels.h"),
    "stage_kernel": ("stage.hip", "stage.h", "hh_device.h"),
    # one psst_adjoint call: the forward kernels' recomputation, the reverse
    # sweep and the contraction, per segment
    "adjoint": ("adjoint.hip", "rk4_wg.hip", "wg_common.h", "hh_device.h", "kernels.h"),
}
# kernel-name substrings whose dispatches make up one launch of each entry
KERNEL_NAMES = {"rk4_wg_kernel": ("rk4_wg_kernel", "rk4_lg_kernel"),
                "stage_kernel": ("stage_kernel",)}


def kernel_sha(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_1906_03958_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


# the workload a kernel's plain traffic file is taken on; others get their own
PRIMARY_WORKLOAD = {"rk4_wg_kernel": "batched", "stage_kernel": "large"}


def traffic_file(kernel, workload=None):
    if workload is None or workload == PRIMARY_WORKLOAD.get(kernel):
        return os.path.join(ROOT, "profiles", f"{kernel}_traffic.txt")
    return os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")


def workload_key(args, workload=None):
    """What a counter figure on file must have been taken on: the workload and
    the sizes that set one launch's work."""
    wl = workload or args.workload
    if wl == "adjoint":
        return {"workload": wl, "trials": args.adjoint_trials, "steps": args.adjoint_steps,
                "K": args.adjoint_K}
    if wl in ("large", "large-sparse"):
        return {"workload": wl}          # one launch is one stage whatever the chunk
    return {"workload": wl, "chunk": args.chunk, "instances": args.instances}


def _longest(rows):
    """Counter values of the longest dispatches (the timed launches, not the
    short tuning runs)."""
    longest = max(d for d, _ in rows)
    return [v for d, v in rows if d > 0.5 * longest]


def write_traffic(args):
    """Per-launch HBM bytes of a kernel from rocprofv3 counters.

    FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled by the
    ratio of the known byte count of a plain device copy to what the same
    counter reads for that copy."""
    kernel, f_csv, w_csv, cf_csv, cw_csv = args.write_traffic
    ref = args.copy_calibration * (1 << 20) if args.copy_calibration else (1 << 30)
    cf = [v for _, v in _counter_rows(cf_csv, "copyBuffer", "FETCH_SIZE")]
    cw = [v for _, v in _counter_rows(cw_csv, "copyBuffer", "WRITE_SIZE")]
    kf = float(ref) / (1024.0 * float(np.median(cf)))
    kw = float(ref) / (1024.0 * float(np.median(cw)))
    # a launch's bytes: for each kernel of the launch, the mean over its
    # longest dispatches, summed over the kernels
    fetch = write = 0.0
    nf = 0
    for kname in KERNEL_NAMES[kernel]:
        fv, n_f = _per_launch(f_csv, kname, "FETCH_SIZE")
        wv, _ = _per_launch(w_csv, kname, "WRITE_SIZE")
        fetch += fv * 1024 * kf
        write += wv * 1024 * kw
        nf = max(nf, n_f)
    f = [None] * nf
    out = dict(kernel=kernel, kernel_source_sha=kernel_sha(kernel), **workload_key(args),
               fetch_bytes_per_launch=fetch, write_bytes_per_launch=write,
               hbm_bytes_per_launch=fetch + write, fetch_scale=kf, write_scale=kw,
               launches=len(f), copy_reference_bytes=ref)
    with open(traffic_file(kernel, args.workload), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))


# float64 flop counters: the VALU ones add the flops of each wavefront
# instruction once (an fma counts 2), so the lane total is 64 times their sum;
# the matrix-core one counts in units of 512 flops
FLOP_COUNTERS = {"SQ_INSTS_VALU_FLOPS_FP64": 64.0, "SQ_INSTS_VALU_FLOPS_FP64_TRANS": 64.0,
                 "SQ_INSTS_VALU_MFMA_MOPS_F64": 512.0}


def write_flops(args):
    """Per-launch float64 flops of a kernel from rocprofv3 counters (one run
    holding SQ_INSTS_VALU_FLOPS_FP64, SQ_INSTS_VALU_FLOPS_FP64_TRANS and, when
    present, SQ_INSTS_VALU_MFMA_MOPS_F64), mean over the longest dispatches."""
    kernel, csv_path = args.write_flops
    per = {}
    for c in FLOP_COUNTERS:
        rows = _counter_rows(csv_path, kernel, c)
        if rows:
            per[c] = float(np.mean(_longest(rows)))
    total = sum(FLOP_COUNTERS[c] * v for c, v in per.items())
    out = dict(kernel=kernel, kernel_source_sha=kernel_sha(kernel), **workload_key(args),
               fp64_flops_per_launch=total, counters=per,
               scale={c: FLOP_COUNTERS[c] for c in per})
    with open(os.path.join(ROOT, "profiles", f"{kernel}_{args.workload}_flops.txt"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))


def write_adjoint_flops(args):
    """float64 flops of one psst_adjoint call of the adjoint workload from
    rocprofv3 counter files of `bench.py --workload adjoint` runs: the VALU
    counters (SQ_INSTS_VALU_FLOPS_FP64, _TRANS; x 64 lanes) and the
    matrix-core counter (SQ_INSTS_VALU_MFMA_MOPS_F64; x 512) summed over the
    reverse and contraction dispatches and over the forward kernels' short
    recomputation dispatches (the long forward runs of the workload are left
    out), divided by the number of adjoint calls (reverse dispatches / segments)."""
    valu_csv, mfma_csv = args.write_adjoint_flops
    segs = -(-args.adjoint_steps // args.adjoint_K)
    per = {}
    calls = None
    for path, counters in ((valu_csv, ("SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU_FLOPS_FP64_TRANS")),
                           (mfma_csv, ("SQ_INSTS_VALU_MFMA_MOPS_F64",))):
        for c in counters:
            tot = 0.0
            for kname in ("adjoint_reverse", "adjoint_contract"):
                rows = _counter_rows(path, kname, c)
                tot += sum(v for _, v in rows)
                if kname == "adjoint_reverse" and rows:
                    calls = len(rows) // segs
            fwd = _counter_rows(path, "rk4_", c)
            if fwd:
                longest = max(d for d, _ in fwd)
                tot += sum(v for d, v in fwd if d < 0.1 * longest)
            per[c] = tot
    total = sum(FLOP_COUNTERS[c] * v for c, v in per.items()) / calls
    out = dict(kernel="adjoint", kernel_source_sha=kernel_sha("adjoint"),
               **workload_key(args, "adjoint"), fp64_flops_per_launch=total,
               counters_summed_over_calls=per, calls=calls,
               scale={c: FLOP_COUNTERS[c] for c in per})
    with open(os.path.join(ROOT, "profiles", "adjoint_adjoint_flops.txt"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))


def _on_file(path, kernel, key):
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernel_source_sha") != kernel_sha(kernel):
        return None
    if any(t.get(k) != v for k, v in key.items()):
        return None
    return t


def read_flops(kernel, args, workload=None):
    """float64 flops per launch measured for this kernel source and workload,
    or None when no such measurement is on file."""
    key = workload_key(args, workload)
    t = _on_file(os.path.join(ROOT, "profiles", f"{kernel}_{key['workload']}_flops.txt"),
                 kernel, key)
    return t.get("fp64_flops_per_launch") if t else None


def read_traffic(kernel, args, workload=None):
    """HBM bytes per launch measured for this kernel source and workload, or
    None when no such measurement is on file."""
    key = workload_key(args, workload)
    t = _on_file(traffic_file(kernel, key["workload"]), kernel, key)
    return t.get("hbm_bytes_per_launch") if t else None


MFMA_FP32_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6


def run_large(args, torch, psst, W, dev, stream, steps, warmup, chunk, sparse=False):
    """16384 neurons (12288 PN, 4096 LN), dense Bernoulli(0.5) g ~ U(0,0.1) nS
    (sparse: Bernoulli(0.1), g ~ U(0,0.5) nS, the same expected input, stored
    as synapse buckets), 64 stimulus trials; one step = chunk RK4 steps (a
    graph of the method's stage launches per RK4 step).  Returns the
    measurements and the stage kernel's fp32 MFMA roofline."""
    t0 = time.time()
    net = W.config4_network(p=0.1, g_max=0.5) if sparse else W.config4_network()
    B = W.CONFIG4_TRIALS
    i_nA, v0 = W.trial_inputs(4, net.n, B)
    h = psst.network_create(net, storage=psst.STORAGE_SPARSE if sparse else psst.STORAGE_DENSE)
    if args.method != "rk4":
        psst.network_set_tableau(h, W.TABLEAUX[args.method])
    stages = len(W.TABLEAUX[args.method]["b"])
    batch = psst.batch_create([h] * B)
    log(f"large network ready in {time.time() - t0:.1f}s: {psst.batch_describe(batch)}")
    nt = net.n * B
    states = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(v0.ravel()).to(dev), states)
    stim = psst.DeviceStimulus(torch.from_numpy(i_nA.ravel()).to(dev))
    cnt = torch.zeros(nt, dtype=torch.int32, device=dev)
    spk = torch.zeros((nt, SPIKE_CAP), dtype=torch.float32, device=dev)
    rows = chunk // REC_STRIDE
    vtrace = torch.zeros((max(rows, 1), nt), dtype=torch.float32, device=dev)
    step0 = 0

    def bench_step():
        nonlocal step0
        rec = psst.DeviceRecord(vtrace if rows else None, REC_STRIDE, rows, cnt, spk, SPIKE_CAP)
        psst.integrate_batch(batch, states, stim, DT, chunk, step0, rec)
        step0 += chunk

    for _ in range(warmup):
        bench_step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_start = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        bench_step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    psst.batch_poll(batch)
    rk4_steps = chunk * steps
    stage_s = ev0.elapsed_time(ev1) / 1e3 / (stages * rk4_steps)
    _, g_bytes = psst.batch_conductance_bytes(batch)
    if sparse:
        # useful work: one product per synapse and trial; the kernel runs the
        # whole tiles (zeros included) on the matrix cores, as dense storage does
        nnz = int(sum(int(np.count_nonzero(p.mask)) for p in net.pathways))
        flops_stage = 2.0 * nnz * B
        dense_flops = 2.0 * net.n * net.n * B
        achieved = flops_stage / stage_s / 1e12
        traffic = read_traffic("stage_kernel", args, "large-sparse") if args.method == "rk4" else None
        res = {"value": nt * rk4_steps / wall, "unit": "neuron-steps/s",
               "wall_s": wall, "rk4_steps": rk4_steps,
               "ms_per_rk4_step": 1e3 * wall / rk4_steps,
               "workload": "large sparse network: 16384 HH neurons (12288 PN, 4096 LN), "
                           "Bernoulli(0.1) g ~ U(0,0.5) nS, 64 stimulus trials, dt 0.01 ms",
               "launch": psst.batch_describe(batch),
               "roofline": {"bound": "mfma", "achieved": round(achieved, 3),
                            "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(achieved / MFMA_FP32_PEAK_TFLOPS, 4),
                            "traffic": traffic,
                            "traffic_GBps": round(traffic / stage_s / 1e9, 1) if traffic else None,
                            "kernel": "stage_kernel<4,2,1,2,sparse> (conductance tiles built "
                                      "in LDS from synapse buckets, fp32 MFMA GEMM, + fused "
                                      "RK stage)",
                            "avg_launch_ms": round(1e3 * stage_s, 4),
                            "synapses": nnz,
                            "algorithmic_flops_per_launch": flops_stage,
                            "tile_flops_per_launch": dense_flops,
                            "tile_TFLOPs": round(dense_flops / stage_s / 1e12, 2),
                            "tile_frac": round(dense_flops / stage_s / 1e12
                                               / MFMA_FP32_PEAK_TFLOPS, 4),
                            "conductance_bytes_per_launch": g_bytes,
                            "conductance_GBps": round(g_bytes / stage_s / 1e9, 1),
                            "note": "achieved: one product (2 flops) per synapse and trial; "
                                    "tile_*: the n x n x trials products the matrix cores "
                                    f"run; launch time = graph time per step / {stages}"}}
        del batch, h
        return res
    flops_stage = 2.0 * net.n * net.n * B
    achieved = flops_stage / stage_s / 1e12
    # counters on file were taken for classical RK4
    traffic = read_traffic("stage_kernel", args, "large") if args.method == "rk4" else None
    res = {"value": nt * rk4_steps / wall, "unit": "neuron-steps/s",
           "wall_s": wall, "rk4_steps": rk4_steps, "ms_per_rk4_step": 1e3 * wall / rk4_steps,
           "workload": "large dense network: 16384 HH neurons (12288 PN, 4096 LN), "
                       "Bernoulli(0.5) g ~ U(0,0.1) nS, 64 stimulus trials, dt 0.01 ms",
           "launch": psst.batch_describe(batch),
           "roofline": {"bound": "mfma", "achieved": round(achieved, 2),
                        "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / MFMA_FP32_PEAK_TFLOPS, 4),
                        "traffic": traffic,
                        "traffic_GBps": round(traffic / stage_s / 1e9, 1) if traffic else None,
                        "traffic_frac": (round(traffic / stage_s / 1e9 / HBM_PEAK_GBS, 4)
                                         if traffic else None),
                        "kernel": "stage_kernel<4,2,1,2> (fp32 MFMA GEMM, 8 wavefronts, + fused "
                                  "RK stage)",
                        "avg_launch_ms": round(1e3 * stage_s, 4),
                        "algorithmic_flops_per_launch": flops_stage,
                        "conductance_bytes_per_launch": g_bytes,
                        "note": f"launch time = graph time per step / {stages} (the step's "
                                f"{stages} stage launches plus a one-thread counter kernel)"}}
    del batch, h
    return res


def bench_large(args, torch, psst, W, dev, stream, sparse=False):
    """The large network on its own line (--workload large, large-sparse)."""
    r = run_large(args, torch, psst, W, dev, stream, args.steps, args.warmup, args.chunk,
                  sparse=sparse)
    out = {"metric": METRIC, "value": r["value"], "unit": "neuron-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * r["wall_s"] / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 (GEMM) / f64 (RHS)",
           "data": "synthetic",
           "config": {"workload": r["workload"], "rk4_steps_per_step": args.chunk,
                      "method": args.method, "launch": r["launch"]},
           "roofline": r["roofline"]}
    print(json.dumps(out), flush=True)


def bench_streamed(args, torch, psst, W, dev, stream):
    """The batched workload for steps x chunk RK4 steps with V after every
    step (1.1 M floats per step) and spikes streamed to host memory in chunks
    of --chunk steps, against the same steps with records on the device
    every 100 steps."""
    insts = W.config3(args.instances)
    sum_n = int(sum(i.net.n for i in insts))
    nets = [psst.network_create(i.net) for i in insts]
    batch = psst.batch_create(nets)
    v0 = torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    st = torch.zeros(14 * sum_n, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, v0, st)
    n = args.steps * args.chunk
    hv = np.empty((n, sum_n), np.float32)
    hv.fill(0.0)             # resident host memory (first-touch page faults excluded)
    hc = np.zeros(sum_n, np.int32)
    hs = np.zeros((sum_n, SPIKE_CAP), np.float32)
    # warm-up: one chunk streamed (the batch's streaming buffers are pinned
    # once, on first use), then the timed run from the same initial state
    psst.integrate_batch_streamed(batch, st, stim, DT, args.chunk, 0, args.chunk, 1,
                                  hv[:args.chunk], hc, hs, SPIKE_CAP)
    psst.batch_state_init(batch, v0, st)
    hc[:] = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psst.integrate_batch_streamed(batch, st, stim, DT, n, 0, args.chunk, 1, hv, hc, hs,
                                  SPIKE_CAP)
    wall = time.perf_counter() - t0
    # the same steps, records on the device every 100 steps
    st2 = torch.zeros_like(st)
    psst.batch_state_init(batch, v0, st2)
    rows = args.chunk // REC_STRIDE
    vt = torch.zeros((max(rows, 1), sum_n), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        psst.integrate_batch(batch, st2, stim, DT, args.chunk, args.chunk * k,
                             psst.DeviceRecord(vt, REC_STRIDE, rows))
    torch.cuda.synchronize()
    wall2 = time.perf_counter() - t1
    value = sum_n * n / wall
    out = {"metric": METRIC, "value": value, "unit": "neuron-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": 1e3 * wall / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"streamed: the {len(insts)}-network batch, V after every "
                                  f"step and spikes drained to host memory in chunks of "
                                  f"{args.chunk} steps", "rk4_steps": n, "neurons": sum_n,
                      "host_trace_bytes": int(hv.nbytes)},
           "trace_rate_GBps": hv.nbytes / wall / 1e9,
           "device_records_every_100_steps": {"value": sum_n * n / wall2,
                                              "unit": "neuron-steps/s"},
           "streaming_overhead": wall / wall2 - 1.0}
    log(f"streamed: {value:.3e} neuron-steps/s ({hv.nbytes / 1e9:.1f} GB of trace at "
        f"{hv.nbytes / wall / 1e9:.1f} GB/s); device records only: {sum_n * n / wall2:.3e}")
    print(json.dumps(out), flush=True)


def bench_al(args, torch, psst, W, dev, stream):
    """One 120-neuron antennal-lobe-shaped network (90 PN + 30 LN, cholinergic,
    fast- and slow-GABA pathways, pulse-train stimuli) through psst_integrate:
    one persistent launch on one workgroup, --steps x --chunk RK4 steps with
    V recorded every step.  A latency-bound case: the figure is the absolute
    rate of one network."""
    inst = W.config2(0, t_ms=1000.0)
    h = psst.network_create(inst.net)
    n = inst.net.n
    st = torch.zeros(14 * n, dtype=torch.float32, device=dev)
    psst.state_init(h, torch.from_numpy(inst.v0).to(dev), st)
    stim = psst.pack_stimulus([inst.stim], dev)
    total = args.steps * args.chunk
    v = torch.zeros((args.chunk, n), dtype=torch.float32, device=dev)
    psst.integrate(h, st, stim, DT, args.chunk, 0, psst.DeviceRecord(v, 1, args.chunk))
    torch.cuda.synchronize()
    psst.state_init(h, torch.from_numpy(inst.v0).to(dev), st)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        psst.integrate(h, st, stim, DT, args.chunk, k * args.chunk,
                       psst.DeviceRecord(v, 1, args.chunk))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    psst.network_poll(h)
    ms = ev0.elapsed_time(ev1)
    out = {"metric": METRIC, "value": n * total / wall, "unit": "neuron-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": 1e3 * wall / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "one 120-neuron antennal-lobe-shaped network (90 PN + 30 LN; "
                                  "ACh, fast and slow GABA; pulse trains), V every step, "
                                  "psst_integrate", "rk4_steps": total},
           "us_per_rk4_step": 1e3 * ms / total}
    log(f"one AL network: {n * total / wall:.3e} neuron-steps/s, {1e3 * ms / total:.2f} us per step")
    print(json.dumps(out), flush=True)


def bench_adjoint(args, torch, psst, W, dev, stream):
    """Adjoint workload: trials of the 120-neuron network sharing one set of
    conductances; forward with checkpoints every K steps and the V trace,
    MSE loss of the PN traces against targets, psst_adjoint for dL/dg_ij and
    dL/dg_Na, g_K, g_L summed over trials.  Targets: the V traces of the same
    trials at the hidden conductances (a GPU forward run; any targets time
    the same)."""
    B, T, K = args.adjoint_trials, args.adjoint_steps, args.adjoint_K
    hidden, ev, i_nA, v0 = W.config5(B)
    n = ev.n
    stim = psst.DeviceStimulus(torch.from_numpy(i_nA.ravel()).to(dev))
    v0d = torch.from_numpy(v0.ravel()).to(dev)
    nh = psst.network_create(hidden)
    bh = psst.batch_create([nh] * B)
    nt = bh.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(bh, v0d, st)
    target = torch.empty((T, nt), dtype=torch.float32, device=dev)
    psst.integrate_batch(bh, st, stim, DT, T, 0, psst.DeviceRecord(target, 1, T))
    psst.batch_poll(bh)
    del bh, nh
    net = psst.network_create(ev)
    batch = psst.batch_create([net] * B)
    v = torch.empty((T, nt), dtype=torch.float32, device=dev)
    ck = torch.empty(((T + K - 1) // K, 14 * nt), dtype=torch.float32, device=dev)
    pn = torch.zeros(nt, dtype=torch.bool, device=dev)
    for t in range(B):
        pn[t * n:t * n + ev.n_pn] = True
    gg = torch.empty(net.grad_size, dtype=torch.float32, device=dev)
    gna = torch.empty(n, dtype=torch.float32, device=dev)
    gk, gl = torch.empty_like(gna), torch.empty_like(gna)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev2 = torch.cuda.Event(enable_timing=True)
    ev3 = torch.cuda.Event(enable_timing=True)
    res = None
    for rep in range(2):               # first pass warms up (workspace allocation)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        psst.batch_state_init(batch, v0d, st)
        psst.integrate_batch(batch, st, stim, DT, T, 0, psst.DeviceRecord(v, 1, T), ck, K)
        ev1.record(stream)
        dl = torch.where(pn, 2.0 * (v - target) / (B * ev.n_pn * T), torch.zeros_like(v))
        ev2.record(stream)
        psst.adjoint(batch, ck, K, stim, DT, T, 0, dl, gg, gna, gk, gl, per_instance=False)
        ev3.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        psst.batch_poll(batch)
        fwd = ev0.elapsed_time(ev1) / 1e3
        adj = ev2.elapsed_time(ev3) / 1e3
        res = {"workload": f"{B} trials x {n}-neuron network (90 PN + 30 LN, ACh + fast "
                           f"GABA), {T} RK4 steps (dt 0.01 ms), checkpoint every {K} steps; "
                           "MSE of PN traces; gradients w.r.t. g_ij, g_Na, g_K, g_L",
               "adjoint_neuron_steps_per_s": B * n * T / adj,
               "adjoint_steps_per_s": T / adj,
               "adjoint_s": adj, "forward_with_checkpoints_s": fwd,
               "forward_plus_adjoint_s": wall,
               "forward_plus_adjoint_neuron_steps_per_s": B * n * T / wall,
               "grad_norm": float(gg.norm())}
    # roofline of the adjoint kernel: float64 flops per launch from the VALU
    # and matrix-core flop counters of this kernel source (null until taken);
    # beside it the synaptic flops the method needs per step and trial --
    # the recomputed forward's products (4 stages x 2 E) and the reverse
    # stages' transposed products and gradient outer products (4 x 4 E), E =
    # the n^2 entries of the dense matrix -- a lower bound on the work
    fl = read_flops("adjoint", args, "adjoint")
    syn = float(T) * B * (4 * 2 + 4 * 4) * n * n
    tf = fl / adj / 1e12 if fl else None
    res["roofline"] = {"bound": "alu", "achieved": round(tf, 3) if tf else None,
                       "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4) if tf else None,
                       "traffic": None,
                       "kernel": "one psst_adjoint call: per segment the forward kernels' "
                                 "recomputation, adjoint_reverse_kernel, "
                                 "adjoint_contract_kernel (float64 MFMA)",
                       "fp64_flops_per_launch": fl,
                       "synaptic_flops_per_launch": syn,
                       "synaptic_TFLOPs": round(syn / adj / 1e12, 3),
                       "us_per_reverse_step": round(1e6 * adj / T, 2),
                       "note": "peak: float64 vector rate (256 CUs x 128 flop/clk x 2.4 GHz); "
                               "flops per call from SQ_INSTS_VALU_FLOPS_FP64(+_TRANS) x 64 and "
                               "SQ_INSTS_VALU_MFMA_MOPS_F64 x 512 over the call's kernels; "
                               "achieved over the call's time"}
    log(f"adjoint: {res['adjoint_neuron_steps_per_s']:.3e} neuron-steps/s "
        f"({res['adjoint_s']:.2f} s for {T} steps; forward {res['forward_with_checkpoints_s']:.2f} s)")
    return res


def bench_adjoint_line(args, torch, psst, W, dev, stream):
    """The adjoint workload on its own line (--workload adjoint)."""
    r = bench_adjoint(args, torch, psst, W, dev, stream)
    out = {"metric": METRIC, "value": r["adjoint_neuron_steps_per_s"], "unit": "neuron-steps/s",
           "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": 1e3 * r["adjoint_s"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {"workload": r["workload"]},
           "roofline": r["roofline"], "adjoint": r}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed bench steps")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=100, help="RK4 steps per bench step")
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--plain-instances", type=int, default=256)
    ap.add_argument("--plain-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=5000,
                    help="RK4 steps of the oracle sample (also the parity window)")
    ap.add_argument("--cpu-instances", type=int, default=128)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized float32 buffer 5 times (reference kernel "
                         "for scaling HBM counters) and exit")
    ap.add_argument("--read-calibration", type=int, default=0, metavar="MIB",
                    help="only sum a MIB-sized float32 buffer 5 times (a read-only "
                         "reference kernel: checks the copy's FETCH_SIZE factor) and exit")
    ap.add_argument("--write-traffic", nargs=5, metavar=("KERNEL", "FETCH_CSV", "WRITE_CSV",
                                                          "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE counter files of a "
                         "bench run (same --workload/--chunk/--instances) and of a "
                         "--copy-calibration run into profiles/KERNEL_traffic.txt and exit")
    ap.add_argument("--workload", choices=("batched", "large", "large-sparse", "uncoupled",
                                           "sparse", "streamed", "al", "adjoint"),
                    default="batched",
                    help="batched: the 4096-network batch (the default line); large: the "
                         "16384-neuron network x 64 trials on the per-stage MFMA path; "
                         "large-sparse: that network at connection probability 0.1 with "
                         "sparse storage (per-stage synapse buckets); "
                         "uncoupled: the batch with every synapse removed (compute only); "
                         "sparse: the batch at connection probability 0.1, sparse storage; "
                         "streamed: the batch with its full V trace (every step) and spikes "
                         "drained to host memory chunk by chunk; al: one 120-neuron "
                         "antennal-lobe network through psst_integrate (latency-bound); "
                         "adjoint: the adjoint leg alone")
    ap.add_argument("--method", default="rk4",
                    help="explicit Runge-Kutta method of the batched/uncoupled workloads: "
                         "one of the named tableaux (rk4 = the classical kernels)")
    ap.add_argument("--write-adjoint-flops", nargs=2, metavar=("VALU_CSV", "MFMA_CSV"),
                    help="turn rocprofv3 --pmc counter files of two --workload adjoint runs "
                         "(SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_FLOPS_FP64_TRANS; "
                         "SQ_INSTS_VALU_MFMA_MOPS_F64) into profiles/adjoint_adjoint_flops.txt "
                         "and exit")
    ap.add_argument("--write-flops", nargs=2, metavar=("KERNEL", "CSV"),
                    help="turn a rocprofv3 --pmc SQ_INSTS_VALU_FLOPS_FP64 "
                         "SQ_INSTS_VALU_FLOPS_FP64_TRANS counter file of a bench run (same "
                         "--workload/--chunk/--instances) into "
                         "profiles/KERNEL_WORKLOAD_flops.txt and exit")
    ap.add_argument("--adjoint-trials", type=int, default=256)
    ap.add_argument("--adjoint-steps", type=int, default=20000)
    ap.add_argument("--adjoint-K", type=int, default=100)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--large-steps", type=int, default=10,
                    help="timed steps of 20 RK4 steps of the large-network leg")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args()

    if args.write_traffic:
        write_traffic(args)
        return
    if args.write_flops:
        write_flops(args)
        return
    if args.write_adjoint_flops:
        write_adjoint_flops(args)
        return

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(instances are independent: a multi-GPU run would shard them with no "
              "communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1906_03958_amd import psst
    from paper_1906_03958_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": 4 * n, "launches": 5}))
        return
    if args.read_calibration:
        n = args.read_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        tot = 0.0
        for _ in range(5):
            tot += float(a.sum())
        torch.cuda.synchronize()
        print(json.dumps({"read_calibration_bytes": 4 * n, "launches": 5, "sum": tot}))
        return

    if args.workload in ("large", "large-sparse"):
        bench_large(args, torch, psst, W, dev, stream, sparse=args.workload == "large-sparse")
        return
    if args.workload == "streamed":
        bench_streamed(args, torch, psst, W, dev, stream)
        return
    if args.workload == "al":
        bench_al(args, torch, psst, W, dev, stream)
        return
    if args.workload == "adjoint":
        bench_adjoint_line(args, torch, psst, W, dev, stream)
        return

    # ---------------- workload: batched config -----------------------------
    uncoupled = args.workload == "uncoupled"
    sparse = args.workload == "sparse"
    t0 = time.time()
    if uncoupled:
        insts = W.config3_uncoupled(args.instances)
    elif sparse:
        insts = W.config3_sparse(args.instances, 0.1)
    else:
        insts = W.config3(args.instances)
    sizes = np.array([i.net.n for i in insts])
    sum_n = int(sizes.sum())
    sum_n2 = int((sizes.astype(np.int64) ** 2).sum())
    log(f"generated {len(insts)} instances, sum N = {sum_n}, sum N^2 = {sum_n2} "
        f"({time.time() - t0:.1f}s)")
    t0 = time.time()
    nets = [psst.network_create(i.net) for i in insts]
    if args.method != "rk4":
        for h in nets:
            psst.network_set_tableau(h, W.TABLEAUX[args.method])
    batch = psst.batch_create(nets)
    log(f"networks + batch (tuned) in {time.time() - t0:.1f}s: {psst.batch_describe(batch)}")
    v0 = torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    states = torch.zeros(14 * sum_n, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, v0, states)
    rows = args.chunk // REC_STRIDE
    vtrace = torch.zeros((max(rows, 1), sum_n), dtype=torch.float32, device=dev)
    cnt = torch.zeros(sum_n, dtype=torch.int32, device=dev)
    spk = torch.zeros((sum_n, SPIKE_CAP), dtype=torch.float32, device=dev)

    step0 = 0

    def bench_step():
        nonlocal step0
        rec = psst.DeviceRecord(vtrace if rows else None, REC_STRIDE, rows, cnt, spk, SPIKE_CAP)
        psst.integrate_batch(batch, states, stim, DT, args.chunk, step0, rec)
        step0 += args.chunk

    for _ in range(args.warmup):
        bench_step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    launch_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ev0.record(stream)
        bench_step()
        ev1.record(stream)
        ev1.synchronize()
        launch_ms.append(ev0.elapsed_time(ev1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    psst.batch_poll(batch)
    value = sum_n * args.chunk * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps
    avg_launch_s = float(np.mean(launch_ms)) / 1e3
    log(f"batched: {value:.3e} neuron-steps/s, {ms_per_step:.2f} ms per bench step "
        f"({1e3 * ms_per_step / args.chunk:.1f} us per RK4 step)")

    # algorithmic bytes per launch under the library's own placement of the
    # conductances (reported by the library): columns kept in LDS are read
    # once per launch, the others once per stage evaluation; plus the state
    # and compensation words in and out (112 B per neuron), the per-neuron
    # parameters and constant current (32 B), the spike counters (8 B) and
    # the V rows recorded (4 B per neuron per row)
    stages = len(W.TABLEAUX[args.method]["b"])
    g_res, g_str = psst.batch_conductance_bytes(batch)
    other_bytes = sum_n * (112 + 32 + 8 + 4 * rows)
    bytes_per_launch = g_res + stages * args.chunk * g_str + other_bytes
    achieved = bytes_per_launch / avg_launch_s / 1e9
    # the re-stream model: every conductance read at every stage (16 sum N^2
    # per RK4 step) plus 80 sum N of state per step -- an upper bound on what
    # the method could move, exceeded where conductances stay in LDS
    restream = (4 * stages * sum_n2 + 80 * sum_n) * args.chunk
    traffic = read_traffic("rk4_wg_kernel", args)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "rk4_wg_kernel (batched persistent RK4)",
                "avg_launch_ms": round(1e3 * avg_launch_s, 3),
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "conductance_bytes": {"resident_once_per_launch": g_res,
                                      "streamed_per_stage": g_str,
                                      "stages_per_launch": stages * args.chunk},
                "restream_model_bytes_per_launch": restream,
                "restream_model_GBps": round(restream / avg_launch_s / 1e9, 1)}
    if traffic:
        # the counted bytes over the same launch time
        roofline["traffic_GBps"] = round(traffic / avg_launch_s / 1e9, 1)
        roofline["traffic_frac"] = round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)
    if sparse:
        # sparse rows: 8 bytes (column, g) per synapse per stage instead of 4
        # per matrix entry; the same instances with dense storage alongside
        nnz = sum(int(sum((p.mask != 0).sum() for p in i.net.pathways)) for i in insts)
        roofline["traffic"] = None
        roofline["kernel"] = "rk4_wg_kernel (batched persistent RK4, sparse rows)"
        roofline["synapses"] = nnz
        roofline["synapse_bytes_per_stage"] = 8 * nnz
        dnets = [psst.network_create(i.net, storage=psst.STORAGE_DENSE) for i in insts]
        dbatch = psst.batch_create(dnets)
        dst = torch.zeros_like(states)
        psst.batch_state_init(dbatch, v0, dst)
        psst.integrate_batch(dbatch, dst, stim, DT, args.chunk, 0)
        torch.cuda.synchronize()
        ev0.record(stream)
        for k in range(args.steps):
            psst.integrate_batch(dbatch, dst, stim, DT, args.chunk, (k + 1) * args.chunk)
        ev1.record(stream)
        ev1.synchronize()
        dms = ev0.elapsed_time(ev1) / args.steps
        roofline["dense_storage_same_instances"] = {
            "value": sum_n * args.chunk / (dms / 1e3), "avg_launch_ms": round(dms, 3)}
        log(f"same instances, dense storage: {roofline['dense_storage_same_instances']['value']:.3e}"
            " neuron-steps/s")
        del dbatch, dnets
    if uncoupled:
        # no conductances: the float64 right-hand side is the work; flops per
        # launch come from the float64 VALU flop counters of this kernel
        fl = read_flops("rk4_wg_kernel", args)
        tf = fl / avg_launch_s / 1e12 if fl else None
        roofline = {"bound": "alu", "achieved": round(tf, 3) if tf else None,
                    "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4) if tf else None,
                    "traffic": None, "kernel": "rk4_wg_kernel (batched persistent RK4)",
                    "avg_launch_ms": round(1e3 * avg_launch_s, 3),
                    "fp64_flops_per_launch": fl,
                    "note": "peak: float64 vector rate of the chip (256 CUs x 128 flop/clk "
                            "x 2.4 GHz); flops per launch from SQ_INSTS_VALU_FLOPS_FP64 "
                            "(+_TRANS), null until measured for this kernel source"}

    # ---------------- plain form: one network per launch ------------------
    plain = None
    if not args.no_plain and not uncoupled and not sparse:
        pick = stratified(sizes, min(args.plain_instances, len(insts)))
        tot_ns, tot_t = 0, 0.0
        for b in pick:
            inst, net = insts[b], nets[b]
            st = torch.zeros(14 * inst.net.n, dtype=torch.float32, device=dev)
            psst.state_init(net, torch.from_numpy(inst.v0).to(dev), st)
            s1 = psst.pack_stimulus([inst.stim], dev)
            psst.integrate(net, st, s1, DT, 10, 0)
            torch.cuda.synchronize()
            ev0.record(stream)
            psst.integrate(net, st, s1, DT, args.plain_steps, 10)
            ev1.record(stream)
            ev1.synchronize()
            tot_t += ev0.elapsed_time(ev1) / 1e3
            tot_ns += inst.net.n * args.plain_steps
        plain = {"value": tot_ns / tot_t, "unit": "neuron-steps/s",
                 "sample": f"{len(pick)} instances stratified by size, {args.plain_steps} RK4 "
                           "steps each, one psst_integrate launch per network"}
        log(f"plain: {plain['value']:.3e} neuron-steps/s")

    adjoint = None if (args.no_adjoint or uncoupled or sparse) else \
        bench_adjoint(args, torch, psst, W, dev, stream)

    # ---------------- the large network (per-stage MFMA path), short ------
    large = None
    if not (args.no_large or uncoupled or sparse) and args.method == "rk4":
        large = run_large(args, torch, psst, W, dev, stream, args.large_steps, 2, 20)
        log(f"large network: {large['value']:.3e} neuron-steps/s, MFMA "
            f"{large['roofline']['achieved']} TFLOP/s ({large['roofline']['frac']} of peak)")

    # ---------------- CPU baseline (oracle) and parity spot check ---------
    cpu = None
    parity = None
    if not args.no_cpu:
        import oracle
        pick = stratified(sizes, min(args.cpu_instances, len(insts)))
        sub = [insts[b] for b in pick]
        threads = min(os.cpu_count() or 1, 16)
        t0 = time.perf_counter()
        otab = None if args.method == "rk4" else W.TABLEAUX[args.method]
        res = oracle.run_many(sub, args.cpu_steps, dt=float(np.float32(DT)), rec_stride=10, threads=threads,
                              tableau=otab)
        ct = time.perf_counter() - t0
        ns = sum(i.net.n for i in sub) * args.cpu_steps
        cpu = {"value": ns / ct, "unit": "neuron-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(sub)} instances stratified by size, {args.cpu_steps} RK4 steps "
                         f"each ({ct:.1f} s wall on {threads} threads)"}
        # one thread on a smaller sample, and the host it ran on
        sub1 = sub[::8]
        steps1 = max(args.cpu_steps // 2, 1)
        t0 = time.perf_counter()
        oracle.run_many(sub1, steps1, dt=DT, rec_stride=0, threads=1, tableau=otab)
        ct1 = time.perf_counter() - t0
        cpu["value_1thread"] = sum(i.net.n for i in sub1) * steps1 / ct1
        cpu["sample_1thread"] = f"{len(sub1)} of those instances, {steps1} RK4 steps, 1 thread"
        model = ""
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        cpu["host"] = {"cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
                       "model": model}
        log(f"cpu oracle: {cpu['value']:.3e} neuron-steps/s on {threads} threads, "
            f"{cpu['value_1thread']:.3e} on 1 thread")
        # same instances from their initial state on the GPU, V every 10 steps
        states2 = torch.zeros_like(states)
        psst.batch_state_init(batch, v0, states2)
        r2 = args.cpu_steps // 10
        vt2 = torch.zeros((r2, sum_n), dtype=torch.float32, device=dev)
        psst.integrate_batch(batch, states2, stim, DT, args.cpu_steps, 0,
                             psst.DeviceRecord(vt2, 10, r2))
        psst.batch_poll(batch)
        vt2 = vt2.cpu().numpy()
        worst = 0.0
        for b, (r, _) in zip(pick, res):
            a0, a1 = batch.offsets[b], batch.offsets[b + 1]
            worst = max(worst, float(np.abs(vt2[:, a0:a1] - r["v"]).max()))
        parity = {"max_abs_dV_mV": worst, "tolerance_mV": 1e-3,
                  "window_ms": args.cpu_steps * DT, "instances": len(pick),
                  "pass": bool(worst <= 1e-3)}
        log(f"parity spot check: max|dV| = {worst:.3e} mV over {args.cpu_steps * DT} ms")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "neuron-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage": "f32 (state as value+compensation pairs; conductances as given)",
        "data": "synthetic",
        "config": {"workload": (f"uncoupled: {len(insts)} batched instances of 60-480 HH "
                                "neurons with no synapses, I ~ U(0,2) nA, dt 0.01 ms")
                   if uncoupled else
                   (f"sparse: {len(insts)} independent antennal-lobe-shaped HH networks, "
                    "60-480 neurons, Bernoulli(0.1) ACh + fast-GABA synapses, "
                    "g ~ U(0,2.5) nS x LogNormal(0,0.1), sparse storage, dt 0.01 ms")
                   if sparse else
                   (f"batched: {len(insts)} independent antennal-lobe-shaped HH "
                    "networks, 60-480 neurons (PN:LN 3:1), Bernoulli(0.5) ACh + "
                    "fast-GABA synapses, g ~ U(0,0.5) nS x LogNormal(0,0.1), "
                    "I ~ U(0,2) nA, dt 0.01 ms"),
                   "instances": len(insts), "neurons": sum_n, "rk4_steps_per_step": args.chunk,
                   "method": args.method,
                   "dt_ms": DT, "recording": f"spikes + V every {REC_STRIDE} steps",
                   "launch": psst.batch_describe(batch)},
        "plain": plain,
        "batched_over_plain": (value / plain["value"]) if plain else None,
        "parity": parity,
        "adjoint": adjoint,
        "large_network": large,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
