"""The host layer of libri (argument checks, workspace layouts, the batched
plan, status reporting) under AddressSanitizer and UBSan: the library's
sources with sanitized host code, linked with tests/host_sanitize_driver.cpp,
run on this machine without a GPU.  Any sanitizer report (including leaks)
fails the run."""
import os
import subprocess

import pytest


def test_host_layer_under_asan_and_ubsan():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("runs on a host without a GPU (the driver hands host buffers to the library)")
    from paper_2407_19614_amd.build import build_host_sanitized
    exe = build_host_sanitized()
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host layer checks passed" in r.stdout
