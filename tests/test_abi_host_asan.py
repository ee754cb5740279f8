"""The host-side ABI checks (tests/test_abi_host.py: argument validation,
workspace sizes, error paths; no kernel launch) rerun in a child process
against librd_asan.so, whose C++ host code is built with AddressSanitizer,
so an out-of-bounds or use-after-free access in the validation, workspace
layout or planning code aborts the run."""
import os
import subprocess
import sys

from paper_1309_1720_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_checks_under_address_sanitizer():
    lib = build.build_asan()
    env = dict(os.environ, RD_LIBRARY=lib, LD_PRELOAD=build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1:protect_shadow_gap=0")
    probe = subprocess.run([sys.executable, "-c",
                            "import paper_1309_1720_amd as rd; rd.lib(); print(rd.LIB_PATH); "
                            "print(any('asan' in l for l in open('/proc/self/maps')))"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert probe.stdout.split() == [lib, "True"], probe.stdout
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi_host.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    print(res.stdout[-3000:], res.stderr[-3000:])
    assert res.returncode == 0
    assert "AddressSanitizer" not in res.stderr
    assert " passed" in res.stdout
