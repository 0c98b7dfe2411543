"""The C-ABI library loads and exports every function include/*.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(only=None):
    """Functions declared by the C-ABI headers (those with an extern "C"
    block; libm_hip_device.h holds device functions only and exports
    nothing), optionally of one header only."""
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h") or (only is not None and h != only):
            continue
        with open(os.path.join(ROOT, "include", h)) as fh:
            if 'extern "C"' not in fh.read():
                continue
        out = subprocess.run(["gcc", "-E", "-P", os.path.join(ROOT, "include", h)],
                             check=True, capture_output=True, text=True).stdout
        names |= set(re.findall(r"\b(libm_hip_\w+)\s*\(", out))
    return names


# libm_hip_host.h declares the host library's entry point (and includes
# libm_hip.h, whose names the GPU library exports)
HOST_ONLY = {"libm_hip_host_eval", "libm_hip_host_fmod_steps"}


def test_header_declares_the_expected_surface():
    names = _declared()
    assert "libm_hip_sin_u10_f64" in names
    assert "libm_hip_fmod_f32" in names
    assert "libm_hip_eval" in names
    assert len(names) >= 70


def test_library_exports_every_declared_symbol():
    import paper_2001_09258_amd as L
    path = L.library_path()
    if not os.path.exists(path):
        pytest.fail("libm_hip.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    assert _declared("libm_hip_host.h") - _declared("libm_hip.h") == HOST_ONLY
    missing = [n for n in sorted(_declared() - HOST_ONLY) if not hasattr(lib, n)]
    assert not missing, missing


def test_host_library_exports_its_entry_point_and_validates():
    import paper_2001_09258_amd as L
    path = L.host_library_path()
    if not os.path.exists(path):
        pytest.fail("libm_hip_host.so is not built (run __graft_entry__.build())")
    lib = L.load_host()
    assert all(hasattr(lib, n) for n in HOST_ONLY)
    f = lib.libm_hip_host_eval
    assert f(L.FN_CODES["exp"], 0, 0, None, None, None, 0) == 0        # n == 0
    assert f(L.FN_CODES["exp"], 0, 0, None, None, None, 5) == 1        # NULL, n > 0
    assert f(L.FN_CODES["exp"], 0, 2, None, None, None, 5) == 2        # bf16: unsupported
    assert f(L.FN_CODES["exp"], 1, 0, None, None, None, 5) == 2        # exp u35: not served
    assert f(99, 0, 0, None, None, None, 5) == 2


def test_binding_mirrors_entry_points():
    import paper_2001_09258_amd as L
    declared = _declared()
    for fn, v, dt, name in L.all_entry_points():
        assert name in declared, name
        assert callable(getattr(L, name))


def test_host_side_validation_without_gpu():
    """NULL pointers with n > 0 are rejected before any HIP call; n == 0 is
    a no-op.  Neither touches the device."""
    import paper_2001_09258_amd as L
    lib = L.load()
    assert lib.libm_hip_exp_u10_f64(None, None, 0, None) == 0
    assert lib.libm_hip_exp_u10_f64(None, None, 10, None) == 1
    assert b"NULL" in lib.libm_hip_last_error()
    assert lib.libm_hip_eval(99, 0, 0, None, None, None, 0, None) in (0, 2)


def test_tune_cache_roundtrip_without_gpu(tmp_path):
    """The tuning table loads from and saves to its text format (no device
    work is involved)."""
    import paper_2001_09258_amd as L
    src = tmp_path / "in.txt"
    src.write_text("24 20 512 2\n24 26 128 4\n999999 3 256 1\n24 5 300 1\n24 7 256 3\n")
    L.tune_reset()
    L.tune_load(str(src))
    dst = tmp_path / "out.txt"
    L.tune_save(str(dst))
    lines = sorted(dst.read_text().split("\n"))
    assert [l for l in lines if l] == ["24 20 512 2", "24 26 128 4"]   # invalid rows dropped
    L.tune_reset()
    L.tune_save(str(dst))
    assert dst.read_text() == ""


def test_device_header_compiles_for_gfx950(tmp_path):
    """include/libm_hip_device.h builds into a user kernel (device code only,
    no GPU needed)."""
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not installed")
    src = tmp_path / "user.hip"
    src.write_text('#include "libm_hip_device.h"\n'
                   "__global__ void k(const double* x, float* y) {\n"
                   "  int i = threadIdx.x;\n"
                   "  y[i] = libm_hip_device::tanh_u10((float)x[i]) +\n"
                   "         (float)libm_hip_device::pow_u10(x[i], 0.5);\n"
                   "}\n")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "--cuda-device-only",
                    "-fsyntax-only", "-I", os.path.join(ROOT, "include"), str(src)],
                   check=True, capture_output=True)


def test_batch_plan_argument_errors_without_a_gpu():
    """Invalid plan arguments are rejected before any HIP call, with the
    message on the library's thread-local error channel."""
    import paper_2001_09258_amd as L
    lib = ctypes.CDLL(L.library_path())
    lib.libm_hip_last_error.restype = ctypes.c_char_p
    lib.libm_hip_batch_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    assert lib.libm_hip_batch_plan_create(ctypes.byref(h), 0, -1) == 1
    assert b"max_requests" in lib.libm_hip_last_error()
    assert lib.libm_hip_batch_last_error() == lib.libm_hip_last_error()
    assert lib.libm_hip_batch_plan_create(ctypes.byref(h), 2000, -1) == 1
    assert lib.libm_hip_batch_plan_create(None, 4, -1) == 1
    assert lib.libm_hip_batch_plan_set_graph(None, 0) == 1
    assert h.value is None
