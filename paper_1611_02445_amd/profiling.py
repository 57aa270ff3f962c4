"""Summaries of rocprofv3 output for the committed performance record.

    python -m paper_1611_02445_amd.profiling trace   <trace_dir> <out.txt> <command...>
    python -m paper_1611_02445_amd.profiling counters <fetch_dir> <write_dir> <copy_fetch_dir> \
        <copy_write_dir> <copy_bytes> <kernel_substring> <grid_size|any> <out.json> <command...>

    python -m paper_1611_02445_amd.profiling table <out.txt> <command> <copy_fetch_dir> <copy_write_dir> \
        <copy_bytes> <pmc_dir>... -- <label>=<kernel_substring>@<grid_size|any> ...

``trace`` turns a ``rocprofv3 --kernel-trace --stats -f csv`` directory into a
per-kernel table (calls, average / min / max duration).  ``counters`` turns
two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of the workload plus the
same two counters read on a plain device copy of known size (copy_bytes read
and copy_bytes written) into HBM bytes per launch: each counter is scaled by
copy_bytes / (the bytes that counter reported for the copy), which calibrates
what the counter actually counts on this GPU.  ``table`` lists the
per-dispatch average of every counter of some ``--pmc`` runs for chosen
kernels.
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def _code_only(text):
    """Source text without comments and blank space: a counter summary stays
    valid when only the comments of the kernels change."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    """Hash of the kernel code (comments ignored); a counter summary is valid
    only for it."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "common.hpp", "kernels.hpp"):
        with open(os.path.join(HERE, "csrc", name), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def _find(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return hits[0]


def trace_table(trace_dir):
    """{(kernel name, grid size): (calls, avg_us, min_us, max_us)}: one kernel
    launched on two workloads (different grids) gets two rows."""
    path = _find(trace_dir, "*kernel_trace.csv")
    d = defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            d[(r["Kernel_Name"], grid)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return {k: (len(v), sum(v) / len(v), min(v), max(v)) for k, v in d.items()}


def trace_summary(trace_dir, command):
    rows = sorted(trace_table(trace_dir).items(), key=lambda kv: -kv[1][0] * kv[1][1])
    out = [f"# rocprofv3 kernel trace: {command}", "",
           f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'grid':>10}  kernel"]
    for (name, grid), (n, avg, lo, hi) in rows:
        out.append(f"{n:6d} {avg:10.2f} {lo:10.2f} {hi:10.2f} {grid:10d}  {name}")
    return "\n".join(out) + "\n"


def counter_per_dispatch(pmc_dir, counter, kernel_substring, grid=None):
    path = _find(pmc_dir, "*counter_collection.csv")
    vals = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter and kernel_substring in r["Kernel_Name"] and \
                    (grid is None or int(r["Grid_Size"]) == grid):
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise ValueError(f"no {counter} rows for kernels matching {kernel_substring!r} in {path}")
    return sum(vals) / len(vals), len(vals)


def counters_summary(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_bytes, kernel_substring, command,
                     grid=None):
    fetch_kib, nf = counter_per_dispatch(fetch_dir, "FETCH_SIZE", kernel_substring, grid)
    write_kib, nw = counter_per_dispatch(write_dir, "WRITE_SIZE", kernel_substring, grid)
    cfetch_kib, _ = counter_per_dispatch(cfetch_dir, "FETCH_SIZE", "copyBuffer")
    cwrite_kib, _ = counter_per_dispatch(cwrite_dir, "WRITE_SIZE", "copyBuffer")
    fs = copy_bytes / (cfetch_kib * 1024.0)
    ws = copy_bytes / (cwrite_kib * 1024.0)
    hbm = fetch_kib * 1024.0 * fs + write_kib * 1024.0 * ws
    return {
        "kernel": kernel_substring,
        "grid_size": grid,
        "kernel_source_hash": kernel_source_hash(),
        "command": command,
        "fetch_size_kib_per_dispatch": fetch_kib,
        "write_size_kib_per_dispatch": write_kib,
        "dispatches": [nf, nw],
        "copy_calibration": {"bytes_read_and_bytes_written_each": copy_bytes, "fetch_size_kib": cfetch_kib,
                             "write_size_kib": cwrite_kib, "fetch_scale": fs, "write_scale": ws},
        "hbm_read_bytes_per_launch": fetch_kib * 1024.0 * fs,
        "hbm_write_bytes_per_launch": write_kib * 1024.0 * ws,
        "hbm_bytes_per_launch": hbm,
    }


def counters_table(pmc_dirs, rows, command, cfetch_dir, cwrite_dir, copy_bytes):
    """Per-dispatch averages of every counter found in the given --pmc runs,
    one line per (label, kernel substring, grid size) row, plus the HBM bytes
    read and written per dispatch (FETCH_SIZE and WRITE_SIZE scaled by the
    copy calibration, as in counters_summary) and the bytes read counted by
    request size (32, 64 and 128-byte L2-to-memory read requests)."""
    names = []
    for d in pmc_dirs:
        with open(_find(d, "*counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] not in names:
                    names.append(r["Counter_Name"])
    fs = copy_bytes / (counter_per_dispatch(cfetch_dir, "FETCH_SIZE", "copyBuffer")[0] * 1024.0)
    ws = copy_bytes / (counter_per_dispatch(cwrite_dir, "WRITE_SIZE", "copyBuffer")[0] * 1024.0)
    out = [f"# rocprofv3 counters per dispatch: {command}",
           f"# HBM MB = FETCH_SIZE (WRITE_SIZE) KiB x 1024 x {fs:.4f} ({ws:.4f}) / 1e6: the scale makes the counter "
           f"read back a {copy_bytes / 2**30:g} GiB device copy's bytes",
           "# read_MB_by_size = (32 n32 + 64 n64 + 128 n128) / 1e6 from the TCC_EA0_RDREQ_{32B,64B,128B} "
           "request counts, where a run holds them", "",
           f"{'row':<28}{'HBM_read_MB':>14}{'HBM_write_MB':>14}{'read_MB_by_size':>17}" +
           "".join(f"{n:>22}" for n in names)]
    for label, sub, grid in rows:
        vals = {}
        for n in names:
            for d in pmc_dirs:
                try:
                    vals[n] = counter_per_dispatch(d, n, sub, grid)[0]
                    break
                except ValueError:
                    continue
        rd = f"{vals['FETCH_SIZE'] * 1024.0 * fs / 1e6:14.1f}" if "FETCH_SIZE" in vals else f"{'-':>14}"
        wr = f"{vals['WRITE_SIZE'] * 1024.0 * ws / 1e6:14.1f}" if "WRITE_SIZE" in vals else f"{'-':>14}"
        sizes = [f"TCC_EA0_RDREQ_{b}B_sum" for b in (32, 64, 128)]
        if all(k in vals for k in sizes):
            by = f"{sum(b * vals[k] for b, k in zip((32, 64, 128), sizes)) / 1e6:17.1f}"
        else:
            by = f"{'-':>17}"
        out.append(f"{label:<28}{rd}{wr}{by}" +
                   "".join(f"{vals[n]:22.1f}" if n in vals else f"{'-':>22}" for n in names))
    return "\n".join(out) + "\n"


def main(argv):
    if len(argv) >= 4 and argv[1] == "trace":
        with open(argv[3], "w") as fh:
            fh.write(trace_summary(argv[2], " ".join(argv[4:])))
        return 0
    if len(argv) >= 11 and argv[1] == "counters":
        grid = int(argv[8]) if argv[8] != "any" else None
        d = counters_summary(argv[2], argv[3], argv[4], argv[5], float(argv[6]), argv[7], " ".join(argv[10:]), grid)
        with open(argv[9], "w") as fh:
            json.dump(d, fh, indent=1)
        return 0
    if len(argv) >= 9 and argv[1] == "table" and "--" in argv:
        cut = argv.index("--")
        dirs = argv[7:cut]
        rows = []
        for spec in argv[cut + 1:]:
            label, rest = spec.split("=", 1)
            sub, grid = rest.rsplit("@", 1)
            rows.append((label, sub, int(grid) if grid != "any" else None))
        with open(argv[2], "w") as fh:
            fh.write(counters_table(dirs, rows, argv[3], argv[4], argv[5], float(argv[6])))
        return 0
    print(__doc__, file=sys.stderr)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv))
