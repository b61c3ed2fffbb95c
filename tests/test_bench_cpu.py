"""bench.py's contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.lstrip().startswith("{")      # no bench line is printed


def _avg_ms(md, row_start):
    """Average ms of the first kernel-trace table row starting with row_start."""
    for line in open(os.path.join(ROOT, "profiles", md)):
        if line.startswith("| " + row_start):
            return float(line.split("|")[3])
    raise AssertionError(f"no row {row_start!r} in {md}")


def test_recorded_rooflines_are_fractions_of_the_peak():
    """The committed counter bytes over the profiled launch times stay at or
    below the 8 TB/s HBM peak (a figure above it would mean the bytes were
    not moved), and the bench's algorithmic figure under the library's
    placement, 369.8 GB per batched launch, does too."""
    import json
    for traffic, md, row in (("rk4_wg_kernel_traffic.txt", "rk4_wg_kernel_batched_4096.md",
                              "rk4_wg_kernel<512"),
                             ("stage_kernel_traffic.txt", "stage_kernel_large_16384.md",
                              "stage_kernel<4"),
                             ("stage_kernel_large-sparse_traffic.txt",
                              "stage_kernel_large_sparse_16384.md", "stage_kernel<4")):
        t = json.load(open(os.path.join(ROOT, "profiles", traffic)))
        ms = _avg_ms(md, row)
        frac = t["hbm_bytes_per_launch"] / (ms / 1e3) / 8e12
        assert 0.0 < frac <= 1.0, (traffic, frac)
    ms = _avg_ms("rk4_wg_kernel_batched_4096.md", "rk4_wg_kernel<512")
    assert 0.0 < 369.8e9 / (ms / 1e3) / 8e12 <= 1.0


def test_per_launch_counters_sum_the_kernels_of_a_launch(tmp_path):
    """A batch launches one kernel per launch group (a kernel name and grid;
    two groups may share a kernel): a launch's counter value is the sum over
    the groups of the run's last launch of each group's mean over its
    dispatches near its longest, leaving out the tuner's shorter runs and the
    groups only the tuner ran."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    ms = 1_000_000        # ns
    rows = [  # kernel, grid, start, end (ns), value
        ("k<256, 2, 32>", 256, 1 * ms, 3 * ms, 99.0),      # tuner: one round
        ("k<512, 1>", 900, 5 * ms, 10 * ms, 99.0),         # tuner: another plan
        ("k<512, 1>", 700, 20 * ms, 25 * ms, 99.0),        # tuner: plan timing, 50 steps
        # two launches of three groups (two share a kernel), run one after another
        ("k<512, 1>", 700, 30 * ms, 40 * ms, 10.0), ("k<512, 1>", 200, 40 * ms, 42 * ms, 3.0),
        ("k<256, 2, 48>", 100, 42 * ms, 46 * ms, 5.0),
        ("k<512, 1>", 700, 50 * ms, 60 * ms, 12.0), ("k<512, 1>", 200, 60 * ms, 62 * ms, 3.0),
        ("k<256, 2, 48>", 100, 62 * ms, 65.9 * ms, 7.0),
        ("other", 1, 0, 5000 * ms, 1e9)]
    path = tmp_path / "c.csv"
    with open(path, "w") as fh:
        fh.write("Kernel_Name,Grid_Size,Counter_Name,Counter_Value,Start_Timestamp,End_Timestamp\n")
        for k, g, a, b, v in rows:
            fh.write(f'"{k}",{g},FETCH_SIZE,{v},{int(a)},{int(b)}\n')
    total, n = bench._per_launch(str(path), "k<", "FETCH_SIZE")
    assert total == 11.0 + 3.0 + 6.0 and n == 2


def test_traffic_on_file_is_keyed_by_workload_and_source(tmp_path):
    """The stage kernel's counter bytes for dense and sparse storage live in
    files of their own, each read back only for its workload, and only while
    the kernel's sources hash to the value recorded with them."""
    import argparse
    import importlib.util
    import json
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    dense = bench.traffic_file("stage_kernel", "large")
    sparse = bench.traffic_file("stage_kernel", "large-sparse")
    assert dense.endswith("stage_kernel_traffic.txt") and sparse != dense
    args = argparse.Namespace(workload="large", chunk=100, instances=4096)
    for path, wl in ((dense, "large"), (sparse, "large-sparse")):
        t = json.load(open(path))
        assert t["workload"] == wl
        if t["kernel_source_sha"] == bench.kernel_sha("stage_kernel"):
            assert bench.read_traffic("stage_kernel", args, wl) == t["hbm_bytes_per_launch"]
    # a record taken on other sources, or on another workload, is not used
    rec = json.load(open(dense))
    cur = dict(rec, kernel_source_sha=bench.kernel_sha("stage_kernel"))
    for t, key, used in ((cur, {"workload": "large"}, True),
                         (cur, {"workload": "large-sparse"}, False),
                         (dict(rec, kernel_source_sha="0" * 16), {"workload": "large"}, False)):
        path = tmp_path / "t.json"
        path.write_text(json.dumps(t))
        assert (bench._on_file(str(path), "stage_kernel", key) is not None) == used
