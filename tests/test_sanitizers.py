"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The library's host sources (geometry, the C ABI's argument checks and plan
set-up, the batch front end) and the C oracle are built with both
sanitizers, every report fatal, and driven in a child process that preloads
the sanitizer runtime.  The child must finish cleanly and give the same
results as the regular builds in this process."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


def _child(call, env):
    code = (f"import sys, json; sys.path[:0] = [{ROOT!r}, {TESTS!r}]; {call[0]}; "
            f"print(json.dumps({call[1]}))")
    e = dict(os.environ)
    e.update(env)
    e["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    e["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-c", code], env=e, cwd=ROOT, capture_output=True,
                       text=True, timeout=900)
    assert r.returncode == 0, f"child exited with {r.returncode}:\n{r.stderr[-6000:]}"
    for mark in ("Sanitizer", "runtime error:"):
        assert mark not in r.stderr, r.stderr[-6000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_library_host_code_is_clean(tmp_path):
    from paper_2204_10871_amd import build as libbuild
    import host_calls
    san = libbuild.build_host_sanitized(str(tmp_path))
    want = json.loads(json.dumps(host_calls.run(libbuild.LIB)))
    got = _child(("import host_calls", f"host_calls.run({san!r})"),
                 {"LD_PRELOAD": libbuild.asan_runtime()})
    assert got.keys() == want.keys()
    for k in want:
        assert got[k] == want[k], k


def test_oracle_is_clean(tmp_path):
    import oracle
    import oracle_calls
    path = oracle.core.build_sanitized(str(tmp_path / "liboracle_san.so"))
    want = json.loads(json.dumps(oracle_calls.run()))
    gcc = lambda name: subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                                      text=True, check=True).stdout.strip()
    got = _child(("import oracle_calls", "oracle_calls.run()"),
                 {"LD_PRELOAD": f"{gcc('libasan.so')}:{gcc('libubsan.so')}",
                  "IRS_ORACLE_LIB": path})
    assert got.keys() == want.keys()
    for k in want:
        assert got[k] == want[k], k
