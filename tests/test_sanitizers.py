"""CPU sanitizer job: the oracle and the library's host-side argument checking under
AddressSanitizer + UndefinedBehaviorSanitizer (any report aborts the run).

* The oracle (lw_oracle.c, gcc -fsanitize=address,undefined) runs every oracle pin
  (tests/test_oracle_*.py, -m "not gpu") in a child process with gcc's libasan preloaded.
* liblw.so rebuilt with its host code sanitized (hipcc -Xarch_host -fsanitize=...; the device
  code is unchanged) runs tests/test_abi.py in a child process with the ASan runtime of
  hipcc's compiler preloaded.

Leak detection is off: the Python interpreter itself keeps allocations alive at exit."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_pytest(files, env_extra, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", *files]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    return out


def test_oracle_pins_under_asan_ubsan(tmp_path):
    import oracle
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not installed")
    lib = oracle.build_sanitized(str(tmp_path / "liblw_oracle_san.so"))
    files = sorted(os.path.relpath(f, ROOT) for f in glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    assert files
    out = _run_pytest(files, {"LD_PRELOAD": oracle.asan_runtime(), "LW_ORACLE_LIBRARY": lib}, timeout=600)
    print(out.strip().splitlines()[-1])


def test_abi_host_validation_under_asan_ubsan(tmp_path):
    from paper_2206_03015_amd import build as hip_build
    try:
        rt = hip_build.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = hip_build.build(sanitize=True, out=str(tmp_path / "liblw_san.so"))
    out = _run_pytest(["tests/test_abi.py"], {"LD_PRELOAD": rt, "LW_LIBRARY": lib}, timeout=600)
    print(out.strip().splitlines()[-1])
