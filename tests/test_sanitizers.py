"""The host code under the address and undefined-behaviour sanitizers: the
library's host side (key generation, serialization, the level scheduler,
the server's admission, budget, failure and cancel logic in simulate mode,
the launch-shape tables) and the CPU oracle are rebuilt with the sanitizers
and the host-side CPU tests run against those builds in a child process
(the sanitizer runtime preloaded, halting on the first report).  The oracle's
long encrypted-circuit tests are left to the full run described in the
design notes; here the oracle runs its arithmetic pins."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUBSET = ["tests/test_server_host.py", "tests/test_abi.py", "tests/test_tune_host.py", "tests/test_oracle_arith.py"]


def test_host_code_under_asan_and_ubsan(tmp_path):
    if not shutil.which("hipcc") or not os.path.exists("/opt/rocm/llvm/bin/clang"):
        pytest.skip("no ROCm compilers")
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    from paper_2407_19871_amd import _build_sanitize as sb
    rt = ob.sanitizer_runtime()
    if rt is None:
        pytest.skip("no shared address-sanitizer runtime")
    lib = sb.build(str(tmp_path))
    orc = ob.build_sanitized(str(tmp_path))
    env = dict(os.environ, LD_PRELOAD=rt, LOCPIR_LIB=lib, LOCPIR_ORACLE_LIB=orc, LOCPIR_NO_TORCH="1",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", *SUBSET, "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out
