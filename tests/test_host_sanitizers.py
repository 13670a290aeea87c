"""The host code of the library (argument validation, context setup and
teardown paths, status and message handling of the C ABI) under
AddressSanitizer and UndefinedBehaviorSanitizer: the ABI tests run against a
build whose host code is instrumented (device code unchanged), with the
sanitizer runtime preloaded and every report fatal.  No GPU is needed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2511_19036_amd"))
import build  # noqa: E402


@pytest.fixture(scope="module")
def sanitized():
    srcs = [os.path.join(build.HERE, s) for s in build.SOURCES]
    newest = max(os.path.getmtime(p) for p in srcs + [os.path.join(ROOT, "include", "cmg.h")])
    if not os.path.exists(build.SAN_LIB) or os.path.getmtime(build.SAN_LIB) < newest:
        build.build(sanitize=True)
    return build.SAN_LIB


def test_abi_tests_pass_under_address_and_ub_sanitizers(sanitized):
    env = dict(os.environ, LD_PRELOAD=build.sanitizer_runtime(), CMG_LIBRARY=sanitized,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                          "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    # the sanitizers were live: the instrumented library references their runtime
    nm = subprocess.run(["nm", "-D", sanitized], capture_output=True, text=True).stdout
    assert "__asan_report" in nm and "__ubsan_handle" in nm
