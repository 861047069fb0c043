"""CPU checks of the C-ABI library: it loads, exports every function that
include/r4d.h declares, and answers the calls that need no device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "r4d.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(r4d_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("r4d_render_forward", "r4d_render_backward", "r4d_create", "r4d_destroy",
                     "r4d_render_forward_f64", "r4d_render_backward_f64", "r4d_l1_loss_grad"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2402_03307_amd as r4d
    lib = ctypes.CDLL(r4d.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(_declared_functions()) == set(r4d.EXPORTED_SYMBOLS)


def test_status_strings_and_defaults():
    import paper_2402_03307_amd as r4d
    lib = r4d.library()
    assert lib.r4d_status_string(0) == b"R4D_OK"
    assert lib.r4d_status_string(-4) == b"R4D_ERR_CAPACITY"
    assert lib.r4d_status_string(-99) == b"R4D_ERR_UNKNOWN"
    s = r4d.default_settings()
    assert s["tile_size"] == 16 and abs(s["alpha_min"] - 1 / 255) < 1e-9
    assert abs(s["T_min"] - 1e-4) < 1e-9 and abs(s["dilation"] - 0.3) < 1e-7


def test_null_arguments_are_rejected_without_a_device():
    import paper_2402_03307_amd as r4d
    lib = r4d.library()
    assert lib.r4d_create(None, 0) == -1
    assert lib.r4d_render_forward(None, None, None, 1, None, None, None, None) == -1
    assert lib.r4d_render_backward(None, None, None, 1, None, None, None, None, None) == -1
    assert lib.r4d_saved_stats(None, 0, None, None, None, None) == -1
    assert lib.r4d_last_error(None) == b""
    lib.r4d_saved_release(None)
    lib.r4d_destroy(None)


def test_build_writes_library_in_package():
    import paper_2402_03307_amd as r4d
    assert os.path.dirname(r4d.LIB_PATH) == os.path.join(ROOT, "paper_2402_03307_amd")
    assert os.path.getsize(r4d.LIB_PATH) > 0


def _host_check_binary():
    """The sanitized host-layer check (paper_2402_03307_amd/build.py), built
    here from the library's objects when it is missing."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_r4d_build", os.path.join(ROOT, "paper_2402_03307_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    if not os.path.exists(mod.HOST_CHECK):
        mod.build(verbose=False)
    return mod.HOST_CHECK


def test_host_layer_under_sanitizers_without_a_device():
    """The C ABI's host layer built with AddressSanitizer and UBSan
    (tests/abi_host_check.cpp, cpu mode): defaults, names, r4d_create's error
    without a device and the refusal of null arguments run without a memory
    error, leak or undefined operation."""
    import subprocess
    exe = _host_check_binary()
    env = dict(os.environ, HIP_VISIBLE_DEVICES="", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, "cpu"], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi_host_check cpu: ok" in r.stdout
    assert "Sanitizer" not in r.stderr, r.stderr
