"""Summaries of rocprofv3 CSV output for the swept2d kernels.

  python -m paper_1602_07558_amd.profiling stats DIR
      per-kernel calls / average / total duration from *_kernel_stats.csv
  python -m paper_1602_07558_amd.profiling grids DIR
      per kernel and grid size, calls and average duration from
      *_kernel_trace.csv (one kernel runs several workloads: their launches
      differ in grid size)
  python -m paper_1602_07558_amd.profiling counters DIR COUNTER [COUNTER ...]
      per-launch averages of --pmc counters for the swept2d stage and
      per-step kernels in DIR
  python -m paper_1602_07558_amd.profiling traffic FETCH_DIR WRITE_DIR OUT [--copy-bytes B]
      HBM bytes per launch of the heat benchmark's kernels (octahedron, bridge
      pair, first upward pyramid, per-step kernel) from two --pmc runs
      (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled by what
      the same counter reads for the plain copy of B bytes that
      `bench.py --profile-pass` runs.
"""
from __future__ import annotations

import csv
import glob
import os
import re
import sys
from collections import defaultdict


def _rows(directory: str, suffix: str):
    for path in sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            yield from csv.DictReader(f)


def kernel_stats(directory: str):
    out = []
    for r in _rows(directory, "kernel_stats.csv"):
        out.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                    "total_ns": float(r["TotalDurationNs"]), "pct": float(r.get("Percentage", 0.0))})
    return out


def short_name(name: str) -> str:
    m = re.search(r"(k[0-9]?_[a-z0-9_]+)<([^()]*)>", name)
    if m:
        args = m.group(2).replace("swept::", "").replace(" ", "")
        return f"{m.group(1)}<{args}>"
    m = re.search(r"(k_[a-z0-9]+)INS_(\d+)(\w+)", name)
    if m:
        return f"{m.group(1)}<{m.group(3)[:int(m.group(2))]}>"
    for key in ("k_copy8", "k_set_base", "k_batch_bump"):
        if key in name:
            return key
    if "copy" in name.lower() or "elementwise" in name.lower():
        return "torch copy"
    return name[:60]


def counter_values(directory: str, counter: str):
    """kernel name -> list of per-dispatch counter totals."""
    per = defaultdict(float)
    names = {}
    for r in _rows(directory, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    out = defaultdict(list)
    for key, v in per.items():
        out[names[key]].append(v)
    return out


def _pick(values: dict, pred):
    got = [v for name, vs in values.items() if pred(name) for v in vs]
    return sum(got) / len(got) if got else None


# Kernels of the heat 1024^2 FP64 benchmark whose HBM traffic is summarised.
HEAT_KERNELS = {
    "oct": lambda n: "k_oct" in n and "Heat64" in n and "66" in n,
    "bridge_pair": lambda n: "k_bridge_pair" in n and "Heat64" in n and "66" in n,
    "up": lambda n: "k_up" in n and "Heat64" in n and "66" in n,
    "plain": lambda n: "k_plain_cols" in n and "Heat64" in n,
}


def _is_copy(n: str) -> bool:
    return ("copy" in n.lower() or "elementwise" in n.lower()) and "k_copy8" not in n


def traffic_summary(fetch_dir: str, write_dir: str, copy_bytes: int):
    """Per kernel: FETCH_SIZE and WRITE_SIZE per launch (KiB, summed over
    channels), scaled to bytes by what the same counter reads for a plain copy
    of copy_bytes (calibration run in the same process)."""
    f = counter_values(fetch_dir, "FETCH_SIZE")
    w = counter_values(write_dir, "WRITE_SIZE")
    f_copy, w_copy = _pick(f, _is_copy), _pick(w, _is_copy)
    if not f_copy or not w_copy:
        raise RuntimeError("counter runs did not contain the calibration copy")
    fs = copy_bytes / (f_copy * 1024.0)
    ws = copy_bytes / (w_copy * 1024.0)
    out = {"copy_fetch_kib": f_copy, "copy_write_kib": w_copy, "fetch_scale": fs, "write_scale": ws}
    for kind, pred in HEAT_KERNELS.items():
        fk, wk = _pick(f, pred), _pick(w, pred)
        if fk is None or wk is None:
            raise RuntimeError(f"counter runs did not contain the {kind} kernel")
        out[f"{kind}.fetch_kib_per_launch"] = fk
        out[f"{kind}.write_kib_per_launch"] = wk
        out[f"{kind}.fetch_bytes_per_launch"] = fk * 1024.0 * fs
        out[f"{kind}.write_bytes_per_launch"] = wk * 1024.0 * ws
    return out


def grid_stats(directory: str):
    """(short kernel name, grid size in workitems) -> [calls, total ns]."""
    out = defaultdict(lambda: [0, 0.0])
    for r in _rows(directory, "kernel_trace.csv"):
        name = r.get("Kernel_Name", "")
        grid = r.get("Grid_Size_X") or r.get("Grid_Size") or "0"
        dur = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        e = out[(short_name(name), int(float(grid)))]
        e[0] += 1
        e[1] += dur
    return out


def main(argv):
    if argv and argv[0] == "grids":
        rows = grid_stats(argv[1])
        for (name, grid), (calls, tot) in sorted(rows.items(), key=lambda kv: -kv[1][1]):
            print(f"{name:40s} grid={grid:9d} calls={calls:7d} avg_us={tot / calls / 1e3:10.2f} "
                  f"total_ms={tot / 1e6:10.3f}")
        return 0
    if argv and argv[0] == "stats":
        for k in sorted(kernel_stats(argv[1]), key=lambda r: -r["total_ns"]):
            print(f"{short_name(k['name']):40s} calls={k['calls']:7d} avg_us={k['avg_ns'] / 1e3:10.2f} "
                  f"total_ms={k['total_ns'] / 1e6:10.3f} pct={k['pct']:6.2f}")
        return 0
    if argv and argv[0] == "counters":
        directory, names = argv[1], argv[2:]
        rows = defaultdict(dict)
        for c in names:
            for k, vals in counter_values(directory, c).items():
                n = short_name(k)
                if re.match(r"k[0-9]?_", n):
                    rows[n][c] = (sum(vals) / len(vals), len(vals))
        print(f"{'kernel':42s} {'launches':>8s} " + " ".join(f"{c:>16s}" for c in names))
        for n in sorted(rows):
            launches = max(v[1] for v in rows[n].values())
            print(f"{n:42s} {launches:8d} " +
                  " ".join(f"{rows[n][c][0]:16.1f}" if c in rows[n] else f"{'-':>16s}" for c in names))
        return 0
    if argv and argv[0] == "traffic":
        fetch_dir, write_dir, out = argv[1], argv[2], argv[3]
        copy_bytes = 64 << 20
        if "--copy-bytes" in argv:
            copy_bytes = int(argv[argv.index("--copy-bytes") + 1])
        t = traffic_summary(fetch_dir, write_dir, copy_bytes)
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import bench
        with open(out, "w") as fo:
            fo.write("# HBM traffic per launch of the heat 1024x1024 FP64 kernels (tile 64): k_oct<Heat64,66,1024,false>\n"
                     "# (downward pyramid + next upward pyramid), k_bridge_pair<Heat64,66,512,false>, k_up<Heat64,66,1024>\n"
                     "# and the per-step kernel k_plain_cols<Heat64,2>, from bench.py --profile-pass\n"
                     "# Commands (from the repository root, one MI355X; each counter in a run of its own; OUTDIR is any\n"
                     "# scratch directory):\n"
                     "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUTDIR/pmc_fetch -o fetch -- "
                     "python3 bench.py --profile-pass\n"
                     "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUTDIR/pmc_write -o write -- "
                     "python3 bench.py --profile-pass\n"
                     "#   python3 -m paper_1602_07558_amd.profiling traffic OUTDIR/pmc_fetch "
                     "OUTDIR/pmc_write OUT\n"
                     "# FETCH_SIZE / WRITE_SIZE are KiB per dispatch; each is scaled by the ratio of the known bytes "
                     "(64 MiB) of the\n# torch copy that --profile-pass runs to what the same counter reads for that "
                     "copy (fetch_scale, write_scale).\n")
            for k, v in t.items():
                fo.write(f"{k}: {v:.6g}\n")
            fo.write(f"kernel_source_sha256_16: {bench.kernel_source_hash()}\n")
        print(open(out).read())
        return 0
    print(__doc__)
    return 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
