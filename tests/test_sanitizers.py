"""Host-side memory and undefined-behaviour checks.

The FP64 oracle is rebuilt with AddressSanitizer and UndefinedBehaviorSanitizer
(clang -fsanitize=address,undefined, no recovery; gcc's AddressSanitizer does not
check loads of `double complex` elements, clang's does) and its whole pin suite is run
against that build in a child process that preloads the ASan runtime; any invalid
access, overflow or UB aborts the child.  Likewise the host side of the HIP
library (descriptor validation, cluster sizes, planning arithmetic that runs before
any device call) is built with the sanitizers on the host pass only (-Xarch_host)
and driven through the C ABI's host-side error paths.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    from oracle import oracle
    return oracle.sanitizer_runtime()


def _env(extra):
    env = dict(os.environ)
    env.update(extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime")
    env = _env({"CDO_SANITIZE": "1", "LD_PRELOAD": rt})
    # build first (the plain-process build of the sanitized library needs no preload)
    subprocess.check_call([sys.executable, "-c", "from oracle import oracle; oracle.build(force=True)"],
                          cwd=ROOT, env=dict(os.environ, CDO_SANITIZE="1"))
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          "tests/test_oracle_pins.py", "-k", "not mlp"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (res.stdout + res.stderr)[-3000:]
    assert res.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail


@pytest.mark.slow
def test_library_host_paths_under_asan_and_ubsan(tmp_path):
    """The ABI tests (header/export checks, every host-side rejection of descriptors,
    cluster sizes and batch shapes) against a build whose host code carries the
    sanitizers.  Without a GPU the device setup after validation reports CDM_ENODEV."""
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime")
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no hipcc")
    out = str(tmp_path / "libcdm_hostsan.so")
    subprocess.check_call([sys.executable, "-c",
                           "from paper_1902_08653_amd import build; build.build(host_sanitize=True, out=%r)" % out],
                          cwd=ROOT)
    env = _env({"CDM_LIB": out, "LD_PRELOAD": rt})
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi.py"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (res.stdout + res.stderr)[-3000:]
    assert res.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
