"""Build the swept2d HIP library for gfx950 in place (hipcc, no JIT cache).

The library holds every kernel and the C ABI declared in include/swept2d.h.
The stage kernels are compiled as one object per scheme and one per batch
launch class (the same sources with different -D settings), in parallel, then
linked with the host files into libswept2d.so.

Flags: -ffp-contract=off keeps every floating-point expression exactly as
written (no fused multiply-add), so results match a plain IEEE evaluation;
packed FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libswept2d.so")
# The LDS bandwidth probe the benchmark reports as the LDS roofline peak (not
# part of the swept2d library).
PROBE_SRC = os.path.join(CSRC, "probe_lds.hip")
PROBE_LIB = os.path.join(HERE, "libswept2d_probe.so")
# A user scheme built against include/swept2d_scheme.hpp and linked with the
# library (the GPU tests register it through swept2d_register_scheme).
PLUGIN_SRC = os.path.join(ROOT, "tests", "plugin", "paper_eq1_scheme.hip")
PLUGIN_LIB = os.path.join(ROOT, "tests", "plugin", "libpaper_eq1_scheme.so")

SCHEMES = ["Heat64", "Wave64", "Euler64", "Hash64", "Incr64", "Push5", "Heat32C", "Wave32C", "Euler32C",
           "Heat32R", "Wave32R", "Hash25x2", "EulerFD64", "EulerFD32C"]
# Batch launch classes: (window pitch, workgroup size).
# negative pitches: rectangular tiles at window pitch 66, 34 and run-time
BATCH_CLASSES = [(66, 1024), (34, 256), (18, 64), (0, 256), (0, 64), (-66, 1024), (-34, 256), (-1, 256)]

SOURCES = [os.path.join(CSRC, f) for f in ("stages_scheme.hip", "stages_batch.hip", "swept2d_kernels.hip",
                                           "swept2d_api.cpp", "swept2d_batch.cpp",
                                           "swept2d_noalloc.hip", "swept3d.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("engine.hpp", "schemes.hpp", "stages.hpp")] + \
    [os.path.join(ROOT, "include", "swept2d.h"), os.path.join(ROOT, "include", "swept3d.h")]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-value",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the swept2d library needs ROCm's hipcc")


def units() -> list[tuple[str, str, list[str]]]:
    """(object name, source, extra flags) of every translation unit."""
    u = [(f"stages_{s.lower()}.o", os.path.join(CSRC, "stages_scheme.hip"), [f"-DSWEPT_SCHEME={s}"])
         for s in SCHEMES]
    u += [(f"batch_{wc}_{nt}.o", os.path.join(CSRC, "stages_batch.hip"),
           [f"-DSWEPT_BATCH_WC={wc}", f"-DSWEPT_BATCH_NT={nt}"]) for wc, nt in BATCH_CLASSES]
    u += [(os.path.splitext(os.path.basename(p))[0] + ".o", p, [])
          for p in SOURCES if os.path.basename(p) not in ("stages_scheme.hip", "stages_batch.hip")]
    return u


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()

    def compile_one(unit):
        name, src, extra = unit
        out = os.path.join(OBJ, name)
        res = subprocess.run([cc, *FLAGS, *extra, "-c", "-o", out, src], capture_output=True, text=True)
        return name, out, res

    jobs = jobs or max(1, min(os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, units()))
    errors = [(n, r) for n, _, r in results if r.returncode != 0]
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(f"[{n}]\n{r.stdout}{r.stderr}" for n, r in errors))
    if verbose:
        for n, _, r in results:
            if r.stderr.strip():
                sys.stderr.write(f"[{n}]\n{r.stderr}")
    tmp = LIB + ".tmp"
    res = subprocess.run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for _, o, _ in results]],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    build_probe(cc)
    build_plugin(cc)
    return LIB


def build_plugin(cc: str | None = None) -> str:
    cc = cc or hipcc()
    tmp = PLUGIN_LIB + ".tmp"
    res = subprocess.run([cc, *FLAGS, "-shared", "-o", tmp, PLUGIN_SRC, "-L" + HERE, "-lswept2d",
                          "-Wl,-rpath,$ORIGIN/../../paper_1602_07558_amd"], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("plugin build failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, PLUGIN_LIB)
    return PLUGIN_LIB


def build_probe(cc: str | None = None) -> str:
    cc = cc or hipcc()
    tmp = PROBE_LIB + ".tmp"
    res = subprocess.run([cc, *FLAGS, "-shared", "-o", tmp, PROBE_SRC], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("probe build failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
