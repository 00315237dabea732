"""Benchmark: grid-point updates per second of the swept rule on one MI355X.

Workload (one bench step): the 1024 x 1024 periodic heat problem, 5-point
FTCS with r = 0.2, initial field of 8 seeded Fourier modes, advanced 20000
time steps with swept2d_advance (FP64). The state is resident in HBM before
timing starts. Alongside, the same workload is timed with the per-step method
(swept2d_plain_advance) and in FP32 with compensated update, and the oracle
(plain C stepper, host cores) is timed on a bounded sample.

Prints one JSON line. `value` is the swept FP64 rate. `roofline` is for the
dominant kernel (the octahedron: downward pyramid fused with the next upward
pyramid), timed per launch with HIP events on the library's stream during the
timed region.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-cpu]
  python bench.py --profile-pass     (short run used under rocprofv3 --pmc)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NX = NY = 1024
TIMESTEPS = 20000
METRIC = "grid-point updates/sec (swept vs plain per-step, FP64 & FP32-comp) + % HBM roofline"
WORKLOAD = ("heat 1024x1024 periodic, 5-point FTCS r=0.2, 20000 steps, "
            "initial field 8 seeded Fourier modes (wavenumbers 1..8, amplitudes U(-1,1))")

# MI355X published peaks.
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
# LDS: 128 bytes per clock per compute unit, 256 CUs at 2.4 GHz.
LDS_PEAK_GBS = 128 * 256 * 2.4
# Algorithmic work of one heat point update (5-point FTCS): flops
# (uW+uE, uN+uS, their sum, 4u, the difference, r*lap, u + r*lap) and the
# LDS bytes of a point update done in LDS: one FP64 read of the point's own
# value and one FP64 write (neighbours come from registers and lane shifts).
HEAT_FLOPS_PER_UPDATE = 7
HEAT_LDS_BYTES_PER_UPDATE = 2 * 8
BATCH_STEPS = 1024

PROFILE_FILE = os.path.join(ROOT, "profiles", "oct_heat1024_fp64_counters.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1602_07558_amd", "csrc", f)
                  for f in ("stages.hpp", "stages_scheme.hip", "schemes.hpp", "engine.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(launch_kind: str = "oct"):
    """HBM bytes per octahedron launch from the committed rocprofv3 counter
    summary, or None when it is missing or the kernels changed since."""
    if not os.path.exists(PROFILE_FILE):
        return None
    vals = {}
    for line in open(PROFILE_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_runs(g, fn, steps, k):
    import torch
    times = []
    for _ in range(k):
        g.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(steps)
        g.synchronize()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return times


def cpu_baseline(budget_s: float = 12.0):
    import oracle
    import swept_inputs as si
    s = si.heat_field(NX, NY, seed=0)
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    oracle.advance_f64(si.HEAT5, s, [si.HEAT_R], 20, threads=threads)
    probe = time.perf_counter() - t0
    steps = max(20, min(TIMESTEPS, int(20 * budget_s / max(probe, 1e-6))))
    t0 = time.perf_counter()
    oracle.advance_f64(si.HEAT5, s, [si.HEAT_R], steps, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": NX * NY * steps / dt, "unit": "point-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"heat 1024x1024 FP64, first {steps} of the 20000 steps, plain C stepper, {threads} threads"}


def other_workloads(sw, si, np):
    """Throughput of the other workloads at their full sizes over a bounded
    number of steps (the step counts of their parity tests are longer): the
    wave 2048^2 and Euler 512^2 grids (swept, FP64 and FP32C) and the
    uneven 256-grid batch (phased launches, model tile sides)."""
    out = {}

    def rate(make, steps, pts):
        g = make()
        g.advance(steps)   # warm-up (graph capture for the batch)
        g.synchronize()
        t0 = time.perf_counter()
        g.advance(steps)
        g.synchronize()
        dt = time.perf_counter() - t0
        tile = g.tile if isinstance(g, sw.Swept2D) else None
        g.close()
        return pts * steps / dt, tile

    s_w = si.wave_field(2048, 2048, seed=0)
    p_w = si.default_params(si.WAVE_LF)
    for prec, name in ((sw.FP64, "fp64"), (sw.FP32C, "fp32c")):
        def mk(prec=prec):
            g = sw.Swept2D(2048, 2048, si.WAVE_LF, p_w, prec=prec)
            g.upload(s_w)
            return g
        v, tile = rate(mk, 1000, 2048 * 2048)
        out[f"wave2048_{name}"] = {"value": v, "unit": "point-updates/s", "steps": 1000, "tile": tile}
    s_e = si.euler_field(512, 512, seed=0)
    p_e = si.default_params(si.EULER_RUS_RK2, s_e)
    for prec, name in ((sw.FP64, "fp64"), (sw.FP32C, "fp32c")):
        def mk(prec=prec):
            g = sw.Swept2D(512, 512, si.EULER_RUS_RK2, p_e, prec=prec)
            g.upload(s_e)
            return g
        v, tile = rate(mk, 500, 512 * 512)
        out[f"euler512_{name}"] = {"value": v, "unit": "point-updates/s (full RK2 steps)", "steps": 500, "tile": tile}
    specs = si.batch_specs(256, seed=0)
    grids = [dict(nx=b["nx"], ny=b["ny"], pde=b["pde"], prec=b["prec"], params=list(si.default_params(b["pde"])))
             for b in specs]
    pts = sum(b["nx"] * b["ny"] for b in specs)

    def mkb():
        b = sw.Swept2DBatch(grids)
        for i, sp in enumerate(specs):
            b.upload(i, si.initial_state(sp["pde"], sp["nx"], sp["ny"], seed=sp["seed"]))
        return b
    v, _ = rate(mkb, BATCH_STEPS, pts)
    out["batch256"] = {"value": v, "unit": "point-updates/s", "steps": BATCH_STEPS, "grids": len(specs),
                       "points": pts, "mode": "phased launches, model tile sides"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--profile-pass", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (the swept decomposition would "
              "give each GPU a block of tiles and exchange only its boundary panels)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1602_07558_amd as sw
    import swept_inputs as si

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    s0 = si.heat_field(NX, NY, seed=0)
    p = si.default_params(si.HEAT5)

    if args.profile_pass:
        # Short run for counter collection: the swept FP64 path plus a plain
        # copy of known size that calibrates the byte counters.
        g = sw.Swept2D(NX, NY, si.HEAT5, p)
        g.upload(s0)
        g.advance(640)
        g.synchronize()
        a = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": True, "tile": g.tile, "copy_bytes": a.numel()}))
        return

    result = {}

    # ---- swept FP64 (value), with per-kernel HIP events on its stream
    g = sw.Swept2D(NX, NY, si.HEAT5, p)
    tile = g.tile
    g.upload(s0)
    for _ in range(args.warmup):
        g.advance(TIMESTEPS)
    t_swept = timed_runs(g, g.advance, TIMESTEPS, args.steps)
    swept_out = g.download()
    # Per-kernel durations from HIP events on the library's stream, in a pass
    # of its own (the events would add gaps to the timed region).
    g.set_timing(True)
    g.advance(TIMESTEPS)
    g.synchronize()
    kern = {r["kind"]: r for r in g.timing()}
    g.set_timing(False)
    g.close()

    # ---- plain per-step FP64 on the same workload (direct launches)
    gp = sw.Swept2D(NX, NY, si.HEAT5, p)
    gp.upload(s0)
    for _ in range(args.warmup):
        gp.plain_advance(TIMESTEPS)
    t_plain = timed_runs(gp, gp.plain_advance, TIMESTEPS, args.steps)
    gp.set_launch_mode(sw.LAUNCH_GRAPH)
    gp.plain_advance(TIMESTEPS)
    t_plain_graph = timed_runs(gp, gp.plain_advance, TIMESTEPS, args.steps)
    gp.upload(s0)
    gp.set_launch_mode(sw.LAUNCH_DIRECT)
    gp.plain_advance(TIMESTEPS * (args.warmup + args.steps))
    plain_out = gp.download()
    gp.close()
    bitwise_equal = bool(np.array_equal(swept_out, plain_out))

    # ---- FP32 with compensated update, swept and plain
    g32 = sw.Swept2D(NX, NY, si.HEAT5, p, prec=sw.FP32C)
    g32.upload(s0)
    for _ in range(args.warmup):
        g32.advance(TIMESTEPS)
    t_s32 = timed_runs(g32, g32.advance, TIMESTEPS, args.steps)
    g32.close()
    g32p = sw.Swept2D(NX, NY, si.HEAT5, p, prec=sw.FP32C)
    g32p.upload(s0)
    for _ in range(args.warmup):
        g32p.plain_advance(TIMESTEPS)
    t_p32 = timed_runs(g32p, g32p.plain_advance, TIMESTEPS, args.steps)
    g32p.close()

    upd = NX * NY * TIMESTEPS
    ms = 1e3 * float(np.median(t_swept))
    rate = lambda ts: upd / float(np.median(ts))

    oct_k = kern["oct"]
    oct_avg_s = oct_k["ms"] * 1e-3 / oct_k["launches"]
    oct_pts = oct_k["points"] / oct_k["launches"]
    flops = oct_pts * HEAT_FLOPS_PER_UPDATE
    achieved = flops / oct_avg_s / 1e12
    traffic = read_traffic()
    lds_gbs = oct_pts * HEAT_LDS_BYTES_PER_UPDATE / oct_avg_s / 1e9

    result = {
        "metric": METRIC,
        "value": rate(t_swept),
        "unit": "point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "nx": NX, "ny": NY, "timesteps": TIMESTEPS, "method": "swept",
                   "tile": tile, "precision": "fp64"},
        "roofline": {
            "bound": "alu",
            "kernel": "k_oct<Heat64,66,1024,false> (downward pyramid + next upward pyramid, ring runs fetched "
                      "from HBM three levels ahead)",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "flops_per_launch": flops,
            "avg_launch_us": oct_avg_s * 1e6,
        },
        "lds_roofline": {"achieved": lds_gbs, "peak": LDS_PEAK_GBS, "unit": "GB/s", "frac": lds_gbs / LDS_PEAK_GBS,
                         "bytes_per_update": HEAT_LDS_BYTES_PER_UPDATE},
        "kernels": {k: {"launches": r["launches"], "avg_us": r["ms"] * 1e3 / r["launches"]} for k, r in kern.items()},
        "plain": {"value": rate(t_plain), "graph_value": rate(t_plain_graph),
                  "ms_per_step": 1e3 * float(np.median(t_plain))},
        "swept_over_plain": rate(t_swept) / rate(t_plain),
        "fp32c": {"swept_value": rate(t_s32), "plain_value": rate(t_p32),
                  "swept_over_fp64_swept": rate(t_s32) / rate(t_swept)},
        "bitwise_equal_swept_plain": bitwise_equal,
    }
    result["other_workloads"] = other_workloads(sw, si, np)
    if not args.skip_cpu:
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
