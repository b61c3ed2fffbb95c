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
    placement, 392.6 GB per batched launch, does too."""
    import json
    for traffic, md, row in (("rk4_wg_kernel_traffic.txt", "rk4_wg_kernel_batched_4096.md",
                              "rk4_wg_kernel<512"),
                             ("stage_kernel_traffic.txt", "stage_kernel_large_16384.md",
                              "stage_kernel<4")):
        t = json.load(open(os.path.join(ROOT, "profiles", traffic)))
        ms = _avg_ms(md, row)
        frac = t["hbm_bytes_per_launch"] / (ms / 1e3) / 8e12
        assert 0.0 < frac <= 1.0, (traffic, frac)
    ms = _avg_ms("rk4_wg_kernel_batched_4096.md", "rk4_wg_kernel<512")
    assert 0.0 < 392.6e9 / (ms / 1e3) / 8e12 <= 1.0
