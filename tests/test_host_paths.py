"""Host paths without a device (validation, planning, null contexts): the
normal build in this process, and the host build with AddressSanitizer and
UBSan in a child process."""
import os
import subprocess
import sys

import pytest

import _host_paths

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib():
    from paper_2608_01746_amd import lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2608_01746_amd import build
        build.build()
    return L


def test_host_paths(lib):
    from paper_2608_01746_amd import api
    _host_paths.run_all(lib, api)


def test_host_paths_under_address_and_ub_sanitizers():
    from paper_2608_01746_amd import build
    try:
        runtime = build.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    path = build.build_host_sanitized()
    env = dict(os.environ, LD_PRELOAD=runtime,
               # the interpreter and torch are not instrumented: their
               # allocations at exit are not this library's leaks
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(HERE, "_host_paths.py"), path], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host paths OK" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
