"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the C-ABI host tests against a libiod whose host code is instrumented, and
the oracle's pin tests against an instrumented oracle. Each runs in a child
process with the sanitizer runtime preloaded; any report fails the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = """
import sys
sys.path.insert(0, {root!r})
import {mod} as M
M.{attr} = {lib!r}
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *{tests!r}]))
"""


def run_child(runtime, mod, attr, lib, tests):
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    env["LD_LIBRARY_PATH"] = os.path.dirname(runtime) + ":" + env.get("LD_LIBRARY_PATH", "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    code = CHILD.format(root=ROOT, mod=mod, attr=attr, lib=lib,
                        tests=[os.path.join(ROOT, "tests", t) for t in tests])
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=1200)
    print(r.stdout[-800:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]


def test_c_abi_host_code_under_sanitizers(tmp_path):
    import host_sanitizers as S
    rt = S.clang_asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime for hipcc's host compiler")
    lib = S.build_libiod(str(tmp_path / "libiod_san.so"))
    run_child(rt, "paper_2207_13175_amd", "LIB_PATH", lib, ["test_capi_host.py"])


def test_oracle_under_sanitizers(tmp_path):
    import host_sanitizers as S
    rt = S.gcc_asan_runtime()
    if rt is None:
        pytest.skip("no gcc ASan runtime")
    lib = S.build_oracle(str(tmp_path / "liborc_san.so"))
    run_child(rt, "oracle", "_LIB", lib,
              ["test_oracle_pins.py", "test_oracle_variants.py", "test_oracle_sensitivity.py"])
