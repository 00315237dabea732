"""Summaries of rocprofv3 CSV output for the swept2d kernels.

  python -m paper_1602_07558_amd.profiling stats DIR
      per-kernel calls / average / total duration from *_kernel_stats.csv
  python -m paper_1602_07558_amd.profiling traffic FETCH_DIR WRITE_DIR OUT [--copy-bytes B]
      HBM bytes per octahedron launch from two --pmc runs (FETCH_SIZE, then
      WRITE_SIZE, in KiB per dispatch), each scaled by what the same counter
      reads for the plain copy of B bytes that `bench.py --profile-pass` runs.
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
    m = re.search(r"(k_[a-z0-9_]+)<([^()]*)>", name)
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


def traffic_summary(fetch_dir: str, write_dir: str, copy_bytes: int):
    f = counter_values(fetch_dir, "FETCH_SIZE")
    w = counter_values(write_dir, "WRITE_SIZE")
    is_oct = lambda n: "k_oct" in n and "Heat64" in n and "66" in n
    is_copy = lambda n: ("copy" in n.lower() or "elementwise" in n.lower()) and "k_copy8" not in n
    f_oct, w_oct = _pick(f, is_oct), _pick(w, is_oct)
    f_copy, w_copy = _pick(f, is_copy), _pick(w, is_copy)
    if None in (f_oct, w_oct, f_copy, w_copy) or not f_copy or not w_copy:
        raise RuntimeError("counter runs did not contain both the octahedron and the copy kernel")
    fs = copy_bytes / (f_copy * 1024.0)
    ws = copy_bytes / (w_copy * 1024.0)
    return {"fetch_kib_per_launch": f_oct, "write_kib_per_launch": w_oct, "copy_fetch_kib": f_copy,
            "copy_write_kib": w_copy, "fetch_scale": fs, "write_scale": ws,
            "fetch_bytes_per_launch": f_oct * 1024.0 * fs, "write_bytes_per_launch": w_oct * 1024.0 * ws}


def main(argv):
    if argv and argv[0] == "stats":
        for k in sorted(kernel_stats(argv[1]), key=lambda r: -r["total_ns"]):
            print(f"{short_name(k['name']):40s} calls={k['calls']:7d} avg_us={k['avg_ns'] / 1e3:10.2f} "
                  f"total_ms={k['total_ns'] / 1e6:10.3f} pct={k['pct']:6.2f}")
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
            fo.write("# HBM traffic of the octahedron kernel k_oct<Heat64,66,1024,false> per launch "
                     "(heat 1024x1024, tile 64, FP64, ring runs fetched from HBM)\n")
            for k, v in t.items():
                fo.write(f"{k}: {v:.6g}\n")
            fo.write(f"kernel_source_sha256_16: {bench.kernel_source_hash()}\n")
        print(open(out).read())
        return 0
    print(__doc__)
    return 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
