"""The shipped batch tuning table (paper_1906_03958_amd/tuning/<arch>.txt)
follows the grammar the library reads, and names only compiled variants."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1906_03958_amd", "tuning", "gfx950.txt")


def _variants():
    """(threads, neurons per thread, register slots) of the per-instance
    kernels in the variant table of rk4_wg.hip."""
    src = open(os.path.join(ROOT, "paper_1906_03958_amd", "csrc", "rk4_wg.hip")).read()
    out = set()
    for bs, npt in re.findall(r"WG[VG]\((\d+), (\d+)\)", src):
        out.add((int(bs), int(npt), 0))
    for bs, npt, s in re.findall(r"WGR\((\d+), (\d+), (\d+)\)", src):
        out.add((int(bs), int(npt), int(s)))
    return out


def test_shipped_table_parses_and_names_compiled_variants():
    variants = _variants()
    classes, plans = {}, []
    for line in open(TABLE):
        tok = line.split()
        if not tok or tok[0].startswith("#"):
            continue
        assert tok[1].startswith("gfx950"), line
        if tok[0] == "class":
            assert len(tok) == 15, line
            c, gen, sparse, gabab, lds, rr = map(int, tok[2:8])
            bs, npt, slots, pbs, pnpt = map(int, tok[8:13])
            t_best, t_plain = map(float, tok[13:15])
            assert 0 <= c < 7 and gen in (0, 1) and sparse in (0, 1) and gabab in (0, 1)
            assert 0 < lds <= 163840 and rr in (0, 1)
            assert (bs, npt, slots) in variants and (pbs, pnpt, 0) in variants
            assert 0 < t_best <= t_plain
            classes[c] = (bs, npt, slots)
        elif tok[0] == "plan":
            mask, nc = int(tok[7]), int(tok[8])
            counts = list(map(int, tok[9:]))
            assert len(counts) == nc
            plans.append((mask, counts))
        else:
            raise AssertionError(line)
    assert classes and plans
    # the 4096-network batch: seven size classes and the lane-group count
    mask, counts = plans[0]
    assert sum(counts) == 4096 and len(counts) == 8
    for c in range(7):
        if mask >> c & 1:
            assert classes[c][2] > 0, "a class switched to register columns has them"
