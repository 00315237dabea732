"""Host-side checks of the C ABI (CPU only: no kernel is launched).

The library must load and export every function include/swept2d.h and
include/swept3d.h declare;
the Python binding must carry the same names; without a GPU, creating a handle
fails with an error message instead of falling back to anything.
"""
import os
import re
import subprocess

import pytest

import paper_1602_07558_amd as sw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in ("swept2d.h", "swept3d.h")]


def declared_functions():
    names = set()
    for path in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names |= set(re.findall(r"\b(swept[23]d_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if sw._build.stale():
        sw._build.build()
    return sw.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("swept2d_create", "swept2d_advance", "swept2d_plain_advance"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", sw.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (swept[23]d_[a-z_]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(lib, n)


def test_binding_names_match_header():
    assert sorted(sw.EXPORTS) == declared_functions()
    for n in declared_functions():
        assert callable(getattr(sw, n))


def test_library_built_for_gfx950_without_contraction():
    flags = sw._build.FLAGS
    assert "--offload-arch=gfx950" in flags
    assert "-ffp-contract=off" in flags
    assert "-packed-fp32-ops" in flags


LLVM = "/opt/rocm/llvm/bin"


def kernel_scratch_sizes(lib_path, workdir):
    """(kernel name, private segment bytes per lane) of every gfx950 kernel in
    a library built here: its device-code section holds one offload bundle
    per object, each unbundled and its kernel metadata read."""
    sec = os.path.join(workdir, "fatbin.bin")
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", ".hip_fatbin=" + sec, lib_path,
                    os.path.join(workdir, "stripped.so")], check=True)
    data = open(sec, "rb").read()
    starts = [m.start() for m in re.finditer(b"__CLANG_OFFLOAD_BUNDLE__", data)] + [len(data)]
    out = []
    for i in range(len(starts) - 1):
        b, co = os.path.join(workdir, f"b{i}.bin"), os.path.join(workdir, f"c{i}.elf")
        open(b, "wb").write(data[starts[i]:starts[i + 1]])
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--input=" + b, "--output=" + co], check=True)
        notes = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", co], capture_output=True, text=True,
                               check=True).stdout
        name = None
        for line in notes.splitlines():
            line = line.strip()
            if line.startswith(".name:"):
                name = line.split(":", 1)[1].strip()
            elif line.startswith(".private_segment_fixed_size:"):
                out.append((name, int(line.split(":", 1)[1])))
    return out


def test_no_kernel_uses_scratch_memory(lib, tmp_path):
    """Every kernel keeps its per-thread arrays in registers: a register
    array indexed by a value known only at run time, or stores to different
    slots merged at a computed index, would put it in scratch memory, which
    costs the latency-bound level loops far more than its bytes."""
    sizes = kernel_scratch_sizes(sw._build.LIB, str(tmp_path))
    assert len(sizes) > 300  # the stage kernels of every scheme and launch class
    assert [k for k in sizes if k[1]] == []


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device error path")
def test_create_without_device_fails_loudly(lib):
    h = lib.swept2d_create(64, 64, 1, sw.HEAT5, 1)
    assert not h
    assert sw.swept2d_last_error()


def test_error_message_is_per_thread(lib):
    """Each thread sees the message of its own last failure: threads whose
    creates fail for different reasons at the same moment each read back
    their own, and a thread that made no failing call reads none."""
    import threading
    start = threading.Barrier(8)
    seen = {}

    def work(i):
        start.wait()
        if i % 2:
            assert not lib.swept2d_create(64, 64, 2, sw.HEAT5, 1)  # wrong nvars for heat
        else:
            assert not lib.swept2d_create(64, 64, 1, 12345, 1)  # unknown pde
        seen[i] = sw.swept2d_last_error()

    def quiet():
        start.wait()
        seen["quiet"] = sw.swept2d_last_error()

    threads = [threading.Thread(target=work, args=(i,)) for i in range(7)] + [threading.Thread(target=quiet)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=60)
    assert seen["quiet"] == ""
    for i in range(7):
        assert seen[i], i
        assert ("nvars" in seen[i]) == bool(i % 2), (i, seen[i])


def test_invalid_pde_shapes_rejected_before_device(lib):
    assert not lib.swept2d_create(64, 64, 2, sw.HEAT5, 1)
    assert "nvars" in sw.swept2d_last_error()
    assert not lib.swept2d_create(64, 64, 1, 999, 1)
    assert "unknown pde" in sw.swept2d_last_error()
    assert not lib.swept2d_create(1, 64, 1, sw.HEAT5, 1)
    assert not lib.swept2d_create(64, 64, 8, sw.EULER_RUS_RK2, 1)


def test_null_handle_calls_return_einval(lib):
    assert lib.swept2d_advance(None, 1) == sw.EINVAL
    assert lib.swept2d_plain_advance(None, 1) == sw.EINVAL
    assert lib.swept2d_set_tile(None, 8) == sw.EINVAL
    assert lib.swept2d_synchronize(None) == sw.EINVAL
    assert lib.swept2d_state_bytes(None) == 0
    lib.swept2d_destroy(None)


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(sw, "_lib", None)
    monkeypatch.setattr(sw, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError):
        sw.load_library()


def test_single_hip_runtime_in_process(lib):
    """torch and the library must share one HIP runtime (torch's), so torch
    streams and tensors passed to the library are valid in its runtime."""
    maps = open("/proc/self/maps").read()
    hip = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(hip) == 1, hip


def test_batch_arguments_rejected_before_device(lib):
    import ctypes
    iv = lambda *v: (ctypes.c_int * len(v))(*v)
    assert not lib.swept2d_batch_create(0, iv(64), iv(64), iv(sw.HEAT5), iv(sw.FP64), None, 0)
    assert "count" in sw.swept2d_last_error()
    assert not lib.swept2d_batch_create(1, iv(64), iv(64), iv(sw.EULER_RUS_RK2), iv(sw.FP64), None, 0)
    assert "not available in a batch" in sw.swept2d_last_error()
    assert not lib.swept2d_batch_create(1, iv(2), iv(64), iv(sw.TEST_HASH), iv(sw.FP64), None, 0)
    assert not lib.swept2d_batch_create(1, iv(64), iv(64), iv(sw.HEAT5), iv(sw.FP64), None, 0)
    assert "parameters" in sw.swept2d_last_error()
    assert lib.swept2d_batch_advance(None, 1) == sw.EINVAL
    assert lib.swept2d_batch_get_tile(None, 0) == sw.EINVAL
    lib.swept2d_batch_destroy(None)


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device error path")
def test_batch_create_without_device_fails_loudly(lib):
    import ctypes
    iv = lambda *v: (ctypes.c_int * len(v))(*v)
    assert not lib.swept2d_batch_create(1, iv(64), iv(64), iv(sw.TEST_HASH), iv(sw.FP64), None, 0)
    assert sw.swept2d_last_error()


def test_user_scheme_table_is_checked_before_any_device_call(lib):
    """A scheme table with another ABI version is rejected (EINVAL) without
    touching a device."""
    ops = sw.SchemeOps(abi=sw.SCHEME_ABI + 1, nvars=1, substeps=1, nparams=0, nv=1, nw=1, vbytes=8)
    import ctypes
    rc = lib.swept2d_register_scheme(ctypes.addressof(ops))
    assert rc == sw.EINVAL
    assert "ABI" in sw.swept2d_last_error()


def test_user_scheme_plugin_builds_and_exports(lib):
    import ctypes
    plug = ctypes.CDLL(sw._build.PLUGIN_LIB)
    assert hasattr(plug, "paper_eq1_register") and plug.paper_eq1_slots() == 5
