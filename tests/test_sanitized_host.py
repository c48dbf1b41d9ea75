"""The host code of the library (tensor structure, plans, execution setup,
network order) under AddressSanitizer and UndefinedBehaviorSanitizer: the
host-side tests run in a child process against a build whose C++ sources
are instrumented (kernels unchanged), and any sanitizer report fails."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_lib_host.py", "tests/test_network.py", "tests/test_tune_cache.py"]


def test_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2401_01921_amd import build as b
    try:
        lib = b.build_sanitized()
        rt = b.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(f"sanitized build unavailable: {e}")
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "BST_LIB": lib,
        "ASAN_OPTIONS": f"detect_leaks=0:log_path={tmp_path}/asan",
        "UBSAN_OPTIONS": f"halt_on_error=1:print_stacktrace=1:log_path={tmp_path}/ubsan",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                       + HOST_TESTS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = sorted(glob.glob(str(tmp_path / "asan*")) + glob.glob(str(tmp_path / "ubsan*")))
    text = "".join(open(p).read()[:4000] for p in reports)
    assert not reports, text
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
