"""The host C++ of the library (argument checks, the FP64 tree build, the
C ABI's ownership and error paths, including injected allocation failures)
under AddressSanitizer and UndefinedBehaviorSanitizer: the host-tree tests
run in a child process that loads the sanitized build.  CPU only."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHECK_LOADED = """
import paper_1005_5384_amd.octgrav as og
og.lib()
maps = open('/proc/self/maps').read()
assert 'libasan' in maps and 'libubsan' in maps, 'sanitizer runtimes not loaded'
assert 'libocgrav_asan.so' in maps and 'libocgrav.so' not in maps, 'wrong library'
print('sanitized library loaded')
"""


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan():
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    from paper_1005_5384_amd import build_sanitized
    build_sanitized.build()
    env = build_sanitized.sanitizer_env()
    env["PYTHONPATH"] = ROOT
    r = subprocess.run([sys.executable, "-c", CHECK_LOADED], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", "tests/test_host_tree.py"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, (r.stdout[-4000:] + r.stderr[-4000:])
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr
