"""Benchmark: grid-point updates per second of the swept rule on one MI355X.

Workload (one bench step): the 1024 x 1024 periodic heat problem, 5-point
FTCS with r = 0.2, initial field of 8 seeded Fourier modes, advanced 20000
time steps with swept2d_advance (FP64). The state is resident in HBM before
timing starts. Alongside, the same workload is timed with the per-step method
(swept2d_plain_advance), in FP32 with compensated update (FP32C: value and
compensation in HBM; FP32R: values alone in HBM, compensations kept in the
LDS windows), and the oracle (plain C stepper, host cores) on a bounded
sample; the other workloads (wave 2048^2, Euler 512^2, the 256-grid batch)
are timed at their full sizes.

Prints one JSON line. `value` is the swept FP64 rate. `roofline` is the HBM
roofline of the dominant kernel (the octahedron: downward pyramid fused with
the next upward pyramid), its launches timed with HIP events on the
library's stream; the LDS and FP64 rooflines of the same kernel sit beside
it, the LDS peak measured on the device.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-cpu]
  python bench.py --profile-pass [--profile-workload heat|euler_fd|heat3d]
                                     (short run used under rocprofv3 --pmc)
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NX = NY = 1024
TIMESTEPS = 20000
WAVE_STEPS = 10000   # the wave and Euler workloads' own step counts
EULER_STEPS = 5000
METRIC = "grid-point updates/sec (swept vs plain per-step, FP64 & FP32-comp) + % HBM roofline"
WORKLOAD = ("heat 1024x1024 periodic, 5-point FTCS r=0.2, 20000 steps, "
            "initial field 8 seeded Fourier modes (wavenumbers 1..8, amplitudes U(-1,1))")

# MI355X published peaks.
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
CLOCK_HZ = 2.4e9
# Algorithmic work of one heat point update (5-point FTCS): flops
# (uW+uE, uN+uS, their sum, 4u, the difference, r*lap, u + r*lap) and the
# LDS bytes of a point update done in LDS: one FP64 read of the point's own
# value and one FP64 write (neighbours come from registers and lane shifts).
HEAT_FLOPS_PER_UPDATE = 7
HEAT_LDS_BYTES_PER_UPDATE = 2 * 8
BATCH_STEPS = 1024
BATCH_LITERAL_STEPS = 50000

PROFILE_FILE = os.path.join(ROOT, "profiles", "heat1024_fp64_hbm_counters.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1602_07558_amd", "csrc", f)
                  for f in ("stages.hpp", "stages_scheme.hip", "schemes.hpp", "engine.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters():
    """Per-kernel HBM bytes per launch from the committed rocprofv3 counter
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
    out = {}
    try:
        for kind in ("oct", "bridge_pair", "up", "plain"):
            out[kind] = float(vals[f"{kind}.fetch_bytes_per_launch"]) + float(vals[f"{kind}.write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
    return out


def heat_panel_bytes(n: int, vb: int = 8) -> dict:
    """Algorithmic HBM bytes per tile and half cycle of the heat stage
    kernels (one value per point): the octahedron reads the ring of its
    downward pyramid (two x-bridge ends of h(h+3) values per row pair, two
    y-bridge ends of h(h-1)) and writes the four strips of its upward pyramid
    (h(n-h+1) values per row pair); the bridge pair reads four pyramid strips
    and writes its own four ends."""
    h = n // 2
    up = 2 * h * (n - h + 1)
    xb = 2 * h * (h + 3)
    yb = 2 * h * (h - 1)
    return {"oct": (2 * xb + 2 * yb + 4 * up) * vb, "bridge_pair": (4 * up + 2 * xb + 2 * yb) * vb}


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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(budget_s: float = 12.0):
    """The oracle on the host: all host cores (threads = nproc) and one
    thread, each on the first steps of the heat workload sized to about
    budget_s seconds."""
    import oracle
    import swept_inputs as si
    s = si.heat_field(NX, NY, seed=0)
    ncores = os.cpu_count() or 1

    def rate(threads, budget):
        t0 = time.perf_counter()
        oracle.advance_f64(si.HEAT5, s, [si.HEAT_R], 5, threads=threads)
        probe = time.perf_counter() - t0
        steps = max(5, min(TIMESTEPS, int(5 * budget / max(probe, 1e-6))))
        t0 = time.perf_counter()
        oracle.advance_f64(si.HEAT5, s, [si.HEAT_R], steps, threads=threads)
        return NX * NY * steps / (time.perf_counter() - t0), steps

    v_all, st_all = rate(ncores, budget_s)
    v_one, st_one = rate(1, budget_s / 2)
    return {"value": v_all, "unit": "point-updates/s", "cores": ncores, "kind": "oracle",
            "sample": f"heat 1024x1024 FP64, first {st_all} of the 20000 steps, plain C stepper, {ncores} threads",
            "cpu_model": cpu_model(), "nproc": ncores,
            "single_thread": {"value": v_one, "unit": "point-updates/s", "cores": 1,
                              "sample": f"first {st_one} steps, 1 thread"}}


def lds_peak():
    """Measured LDS read bandwidth (bytes/s) of the device."""
    import paper_1602_07558_amd.build as b
    if not os.path.exists(b.PROBE_LIB):
        return None
    lib = ctypes.CDLL(b.PROBE_LIB)
    lib.lds_probe_read_bandwidth.restype = ctypes.c_int
    lib.lds_probe_read_bandwidth.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_int)]
    b64, b128, cus = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    if lib.lds_probe_read_bandwidth(ctypes.byref(b64), ctypes.byref(b128), ctypes.byref(cus)) != 0:
        return None
    return {"b64_GBs": b64.value / 1e9, "b128_GBs": b128.value / 1e9, "cus": cus.value,
            "b64_bytes_per_clk_cu": b64.value / (cus.value * CLOCK_HZ),
            "b128_bytes_per_clk_cu": b128.value / (cus.value * CLOCK_HZ)}


def normwise(x, ref):
    import numpy as np
    return max(float(np.abs(x[v] - ref[v]).max() / np.abs(ref[v]).max()) for v in range(ref.shape[0]))


def other_workloads(sw, si, np):
    """Throughput of the other workloads at their full sizes over a bounded
    number of steps (the step counts of their parity tests are longer), with
    the FP32 forms' normwise error against the FP64 result of the same run:
    the wave 2048^2 and Euler 512^2 grids (swept), the paper's Euler
    discretisation on its 1024 x 512 tunnel (swept and per-step), 3D heat on
    128^3 and 192^3 (swept and per-step), heat on 8192^2 (state beyond the
    Infinity Cache: swept and per-step) and the
    uneven 256-grid batches (phased launches, model tile sides)."""
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
        res = g.download() if isinstance(g, sw.Swept2D) else None
        g.close()
        return pts * steps / dt, tile, res

    def final_state(make, steps):
        g = make()
        g.advance(steps)
        res = g.download()
        g.close()
        return res

    # Error against FP64 at the workloads' own step counts (the FP64 swept
    # result is the oracle's, bit for bit).
    s_w = si.wave_field(2048, 2048, seed=0)
    p_w = si.default_params(si.WAVE_LF)
    ref = None
    for prec, name in ((sw.FP64, "fp64"), (sw.FP32C, "fp32c"), (sw.FP32R, "fp32r")):
        def mk(prec=prec):
            g = sw.Swept2D(2048, 2048, si.WAVE_LF, p_w, prec=prec)
            g.upload(s_w)
            return g
        v, tile, _ = rate(mk, 1000, 2048 * 2048)
        rec = {"value": v, "unit": "point-updates/s", "steps": 1000, "tile": tile}
        res = final_state(mk, WAVE_STEPS)
        if ref is None:
            ref = res
        else:
            rec[f"error_vs_fp64_after_{WAVE_STEPS}_steps"] = normwise(res, ref)
        out[f"wave2048_{name}"] = rec
    s_e = si.euler_field(512, 512, seed=0)
    p_e = si.default_params(si.EULER_RUS_RK2, s_e)
    ref = None
    for prec, name in ((sw.FP64, "fp64"), (sw.FP32C, "fp32c")):
        def mk(prec=prec):
            g = sw.Swept2D(512, 512, si.EULER_RUS_RK2, p_e, prec=prec)
            g.upload(s_e)
            return g
        v, tile, _ = rate(mk, 500, 512 * 512)
        rec = {"value": v, "unit": "point-updates/s (full RK2 steps)", "substep_value": 2 * v,
               "steps": 500, "tile": tile}
        res = final_state(mk, EULER_STEPS)
        if ref is None:
            ref = res
        else:
            rec[f"error_vs_fp64_after_{EULER_STEPS}_steps"] = normwise(res[:4], ref[:4])
        out[f"euler512_{name}"] = rec
    # The paper's own Euler discretisation (skew-symmetric central
    # differences, four-stage Runge-Kutta) on its 1024 x 512 tunnel grid.
    s_f = si.initial_state(si.EULER_FD_RK4, 1024, 512, seed=0)
    p_f = si.default_params(si.EULER_FD_RK4)
    ref = None
    for prec, name in ((sw.FP64, "fp64"), (sw.FP32C, "fp32c")):
        fd = {}
        for method in ("swept", "plain"):
            g = sw.Swept2D(1024, 512, si.EULER_FD_RK4, p_f, prec=prec)
            if prec == sw.FP64:
                g.upload(s_f)
            else:
                # the start as the exact pair u - c of the FP64 state, so the
                # error below is that of the compensated arithmetic, not the
                # FP32 rounding of the free stream (upload keeps c = 0)
                hi = s_f.astype(np.float32)
                g.upload_raw(np.concatenate([hi, (hi.astype(np.float64) - s_f).astype(np.float32)]))
            run = g.advance if method == "swept" else g.plain_advance
            run(20)
            g.synchronize()
            t0 = time.perf_counter()
            run(200)
            g.synchronize()
            fd[method] = 1024 * 512 * 200 / (time.perf_counter() - t0)
            fd["tile"] = g.tile
            if method == "swept":
                res = g.download()  # after 220 steps
            g.close()
        rec = {"swept_value": fd["swept"], "plain_value": fd["plain"], "unit": "point-updates/s (full RK4 steps)",
               "swept_substep_value": 4 * fd["swept"], "steps": 200, "tile": fd["tile"],
               "swept_over_plain": fd["swept"] / fd["plain"],
               "note": "50 MB state (12 values per point, 8 bytes each) stays in the Infinity Cache; "
                       "both paths latency-bound"}
        if ref is None:
            ref = res
        else:
            rec["error_vs_fp64_after_220_steps"] = normwise(res[:4], ref[:4])
        out[f"euler_fd_tunnel1024x512_{name}"] = rec
    # The swept rule in 3D: 7-point heat on 128^3 (cube tile 16) and 192^3
    # (tile 12), swept and per-step.
    for L in (128, 192):
        s3 = si.heat3d_field(L, L, L, seed=0)
        r3 = {}
        for method in ("swept", "plain"):
            g = sw.Swept3D(L, L, L, si.HEAT7_3D, [si.HEAT3D_R])
            g.upload(s3)
            run = g.advance if method == "swept" else g.plain_advance
            run(16)
            g.synchronize()
            t0 = time.perf_counter()
            run(64)
            g.synchronize()
            r3[method] = L ** 3 * 64 / (time.perf_counter() - t0)
            r3["tile"] = g.tile
            g.close()
        out[f"heat3d_{L}_fp64"] = {"swept_value": r3["swept"], "plain_value": r3["plain"],
                                   "unit": "point-updates/s", "steps": 64, "tile": r3["tile"],
                                   "swept_over_plain": r3["swept"] / r3["plain"]}
    # Heat 8192^2 FP64 (512 MB of state, beyond the 256 MB Infinity Cache):
    # the per-step kernel's traffic goes to HBM, with the swept rule beside it.
    s_h = si.heat_field(8192, 8192, seed=0)
    p_h = si.default_params(si.HEAT5)
    big = {}
    for method in ("swept", "plain"):
        g = sw.Swept2D(8192, 8192, si.HEAT5, p_h)
        g.upload(s_h)
        run = g.advance if method == "swept" else g.plain_advance
        run(64)
        g.synchronize()
        t0 = time.perf_counter()
        run(256)
        g.synchronize()
        dt = time.perf_counter() - t0
        big[method] = 8192 * 8192 * 256 / dt
        big["tile"] = g.tile
        g.close()
    out["heat8192_fp64"] = {"swept_value": big["swept"], "plain_value": big["plain"], "unit": "point-updates/s",
                            "steps": 256, "tile": big["tile"], "swept_over_plain": big["swept"] / big["plain"],
                            "plain_algorithmic_hbm_GBs": big["plain"] * 16 / 1e9,
                            "note": "512 MB state: the per-step kernel's 16 B per point-update go to HBM"}
    for quantum, steps, key in ((16, BATCH_STEPS, "batch256"), (1, BATCH_LITERAL_STEPS, "batch256_literal")):
        specs = si.batch_specs(256, seed=0, quantum=quantum)
        grids = [dict(nx=b["nx"], ny=b["ny"], pde=b["pde"], prec=b["prec"], params=list(si.default_params(b["pde"])))
                 for b in specs]
        pts = sum(b["nx"] * b["ny"] for b in specs)

        def mkb(specs=specs, grids=grids):
            b = sw.Swept2DBatch(grids)
            for i, sp in enumerate(specs):
                b.upload(i, si.initial_state(sp["pde"], sp["nx"], sp["ny"], seed=sp["seed"]))
            return b
        b = mkb()
        swept_grids = sum(1 for i in range(len(specs)) if b.tile(i) > 0 or b.rect(i) > 0)
        rect_grids = sum(1 for i in range(len(specs)) if b.rect(i) > 0)
        b.advance(BATCH_STEPS)
        b.synchronize()
        t0 = time.perf_counter()
        b.advance(steps)
        b.synchronize()
        dt = time.perf_counter() - t0
        b.close()
        out[key] = {"value": pts * steps / dt, "unit": "point-updates/s", "steps": steps, "grids": len(specs),
                    "points": pts, "swept_grids": swept_grids, "rect_grids": rect_grids, "side_quantum": quantum,
                    "mode": "phased launches, model tile sides"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--profile-pass", action="store_true")
    ap.add_argument("--profile-workload", choices=("heat", "euler_fd", "heat3d"), default="heat")
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
        # Short run for counter collection: the swept FP64 path, per-step
        # launches, and a plain copy of known size that calibrates the byte
        # counters. heat: 1024^2, 20 half cycles and 64 steps; euler_fd: the
        # 1024 x 512 tunnel, 5 half cycles (40 steps) and 8 steps, in FP64 and
        # then in FP32C; heat3d: 128^3, 4 half cycles (32 steps) and 8 steps.
        if args.profile_workload == "euler_fd":
            for prec in (sw.FP32C, sw.FP64):  # the FP64 handle stays open below
                g = sw.Swept2D(1024, 512, si.EULER_FD_RK4, si.default_params(si.EULER_FD_RK4), prec=prec)
                g.upload(si.initial_state(si.EULER_FD_RK4, 1024, 512, seed=0))
                g.advance(40)
                g.plain_advance(8)
                if prec == sw.FP32C:
                    g.synchronize()
                    g.close()
        elif args.profile_workload == "heat3d":
            g = sw.Swept3D(128, 128, 128, si.HEAT7_3D, [si.HEAT3D_R])
            g.upload(si.heat3d_field(128, 128, 128, seed=0))
            g.advance(32)
            g.plain_advance(8)
        else:
            g = sw.Swept2D(NX, NY, si.HEAT5, p)
            g.upload(s0)
            g.advance(640)
            g.plain_advance(64)
        g.synchronize()
        a = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": True, "tile": g.tile, "copy_bytes": a.numel()}))
        return

    upd = NX * NY * TIMESTEPS
    rate = lambda ts: upd / float(np.median(ts))

    # ---- swept FP64 (value)
    g = sw.Swept2D(NX, NY, si.HEAT5, p)
    tile = g.tile
    g.upload(s0)
    for _ in range(args.warmup):
        g.advance(TIMESTEPS)
    t_swept = timed_runs(g, g.advance, TIMESTEPS, args.steps)
    # The FP64 result after exactly 20000 steps (the oracle's bits, by the
    # full-size parity test): the reference for the FP32 forms' error.
    g.upload(s0)
    g.advance(TIMESTEPS)
    ref64 = g.download()
    # Per-kernel durations from HIP events on the library's stream, in a pass
    # of its own (the events would add gaps to the timed region).
    g.set_timing(True)
    g.advance(TIMESTEPS)
    g.synchronize()
    kern = {r["kind"]: r for r in g.timing()}
    g.set_timing(False)
    g.close()

    # ---- plain per-step FP64 on the same workload (direct launches, then a
    # captured graph)
    gp = sw.Swept2D(NX, NY, si.HEAT5, p)
    gp.upload(s0)
    for _ in range(args.warmup):
        gp.plain_advance(TIMESTEPS)
    t_plain = timed_runs(gp, gp.plain_advance, TIMESTEPS, args.steps)
    gp.set_launch_mode(sw.LAUNCH_GRAPH)
    gp.plain_advance(TIMESTEPS)
    t_plain_graph = timed_runs(gp, gp.plain_advance, TIMESTEPS, args.steps)
    gp.set_launch_mode(sw.LAUNCH_DIRECT)
    gp.upload(s0)
    gp.plain_advance(TIMESTEPS)
    plain_out = gp.download()
    gp.set_timing(True)
    gp.plain_advance(200)
    gp.synchronize()
    kern_plain = {r["kind"]: r for r in gp.timing()}["plain"]
    gp.set_timing(False)
    gp.close()
    bitwise_equal = bool(np.array_equal(ref64, plain_out))

    # ---- FP32 forms, swept and plain, with their error after 20000 steps
    fp32 = {}
    for prec, name in ((sw.FP32C, "fp32c"), (sw.FP32R, "fp32r")):
        g32 = sw.Swept2D(NX, NY, si.HEAT5, p, prec=prec)
        g32.upload(s0)
        for _ in range(args.warmup):
            g32.advance(TIMESTEPS)
        t_s = timed_runs(g32, g32.advance, TIMESTEPS, args.steps)
        g32.upload(s0)
        g32.advance(TIMESTEPS)
        err_s = normwise(g32.download(), ref64)
        g32.upload(s0)
        for _ in range(args.warmup):
            g32.plain_advance(TIMESTEPS)
        t_p = timed_runs(g32, g32.plain_advance, TIMESTEPS, args.steps)
        g32.upload(s0)
        g32.plain_advance(TIMESTEPS)
        err_p = normwise(g32.download(), ref64)
        g32.close()
        fp32[name] = {"swept_value": rate(t_s), "plain_value": rate(t_p),
                      "swept_over_fp64_swept": rate(t_s) / rate(t_swept),
                      "error_vs_fp64_swept": err_s, "error_vs_fp64_plain": err_p,
                      "state_bytes_per_value": 8 if prec == sw.FP32C else 4}
    fp32["fp32c"]["form"] = "FP32 value + FP32 compensation in HBM, LDS and panels (swept == plain bitwise)"
    fp32["fp32r"]["form"] = ("FP32 value only in HBM and panels; compensation in the LDS windows within a residency "
                             "(per-step method = plain FP32)")

    # ---- rooflines of the dominant kernel (octahedron) and the per-step kernel
    oct_k = kern["oct"]
    oct_avg_s = oct_k["ms"] * 1e-3 / oct_k["launches"]
    oct_pts = oct_k["points"] / oct_k["launches"]
    ntiles = (NX // tile) * (NY // tile)
    algo = heat_panel_bytes(tile)
    oct_bytes = algo["oct"] * ntiles
    counters = read_counters()
    lds = lds_peak()
    lds_peak_gbs = lds["b64_GBs"] if lds else None
    lds_gbs = oct_pts * HEAT_LDS_BYTES_PER_UPDATE / oct_avg_s / 1e9
    flops = oct_pts * HEAT_FLOPS_PER_UPDATE / oct_avg_s / 1e12
    plain_avg_s = kern_plain["ms"] * 1e-3 / kern_plain["launches"]
    plain_bytes = 2 * 8 * NX * NY
    half_pts = NX * NY * (tile // 2)
    swept_bytes_algo = (algo["oct"] + algo["bridge_pair"]) * ntiles / half_pts
    swept_bytes_cnt = ((counters["oct"] + counters["bridge_pair"]) / half_pts) if counters else None

    result = {
        "metric": METRIC,
        "value": rate(t_swept),
        "unit": "point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * float(np.median(t_swept)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "nx": NX, "ny": NY, "timesteps": TIMESTEPS, "method": "swept",
                   "tile": tile, "precision": "fp64"},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_oct<Heat64,66,1024,false> (downward pyramid + next upward pyramid, ring runs fetched "
                      "from HBM three levels ahead)",
            "achieved": oct_bytes / oct_avg_s / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": oct_bytes / oct_avg_s / 1e9 / HBM_PEAK_GBS,
            "traffic": counters["oct"] if counters else None,
            "algorithmic_bytes_per_launch": oct_bytes,
            "avg_launch_us": oct_avg_s * 1e6,
            "limiter": "none of HBM, LDS or FP64 issue is saturated: per-level latency (LDS round trip, lane "
                       "shifts, the FP64 chain, the workgroup barrier) of one 16-wave workgroup per CU",
        },
        "lds_roofline": {"achieved": lds_gbs, "peak": lds_peak_gbs, "unit": "GB/s",
                         "frac": (lds_gbs / lds_peak_gbs) if lds_peak_gbs else None,
                         "bytes_per_update": HEAT_LDS_BYTES_PER_UPDATE, "peak_measured": lds},
        "alu_roofline": {"achieved": flops, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": flops / FP64_VECTOR_PEAK_TFLOPS, "flops_per_update": HEAT_FLOPS_PER_UPDATE},
        "hbm_bytes_per_point_update": {
            "swept": {"algorithmic": swept_bytes_algo, "counters": swept_bytes_cnt},
            "plain": {"algorithmic": 16.0, "counters": (counters["plain"] / (NX * NY)) if counters else None},
        },
        "kernels": {k: {"launches": r["launches"], "avg_us": r["ms"] * 1e3 / r["launches"]} for k, r in kern.items()},
        "plain": {"value": rate(t_plain), "graph_value": rate(t_plain_graph),
                  "ms_per_step": 1e3 * float(np.median(t_plain)),
                  "roofline": {"bound": "hbm", "kernel": "k_plain_cols<Heat64,2>", "avg_launch_us": plain_avg_s * 1e6,
                               "achieved": plain_bytes / plain_avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": plain_bytes / plain_avg_s / 1e9 / HBM_PEAK_GBS,
                               "traffic": counters["plain"] if counters else None,
                               "note": "the 8 MB state stays in the 256 MB Infinity Cache; traffic counts HBM bytes"}},
        "swept_over_plain": rate(t_swept) / rate(t_plain),
        "fp32": fp32,
        "bitwise_equal_swept_plain": bitwise_equal,
        "counter_summary": os.path.relpath(PROFILE_FILE, ROOT) if counters else None,
    }
    result["other_workloads"] = other_workloads(sw, si, np)
    if not args.skip_cpu:
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
