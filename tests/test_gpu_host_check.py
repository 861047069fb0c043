"""The C ABI's host layer under AddressSanitizer and UBSan on a device
(tests/abi_host_check.cpp, gpu mode; built by paper_2402_03307_amd/build.py
with the sanitizers on host code only): renders of a small synthetic set in
every mode, with and without front lists, at two tile sizes -- all images
bit-identical -- plus saved-state introspection, the L1 loss, argument errors
on a live context and a saved state released after its context, without a
memory error or undefined operation in the host code."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2402_03307_amd", "abi_host_check")

pytestmark = pytest.mark.gpu


def test_host_layer_under_sanitizers_on_a_device():
    assert os.path.exists(EXE), "abi_host_check is built by paper_2402_03307_amd/build.py"
    print("case: abi_host_check gpu (host layer under ASan + UBSan)", flush=True)
    # leaks are not checked here: the HIP runtime keeps allocations until exit
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([EXE, "gpu"], capture_output=True, text=True, timeout=180, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:], flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi_host_check gpu: ok" in r.stdout
    assert "Sanitizer" not in r.stderr, r.stderr
