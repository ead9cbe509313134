"""Sanitizer builds of host code (CPU only): the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer driven through every step variant (tests/native/oracle_sanitize.c),
and the host side of the HIP library's C ABI compiled with the same sanitizers for host code
(its argument checks need no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-fopenmp",
           "-o", str(exe), os.path.join(ROOT, "tests", "native", "oracle_sanitize.c"),
           os.path.join(ROOT, "oracle", "qed_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout, r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "sanitized run" in r.stdout


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not found")
def test_library_host_code_builds_with_sanitizers(tmp_path):
    """The host code of the C ABI (argument checks, plan bookkeeping) compiles with the host-side
    sanitizers; GPU code is built without them (-Xarch_host puts each option on the host pass)."""
    src = os.path.join(ROOT, "paper_2511_08929_amd", "csrc", "qs_step.hip")
    out = tmp_path / "qs_step_host_sanitized.o"
    cmd = ["/opt/rocm/bin/hipcc", "-c", "-O1", "-std=c++17", "--offload-arch=gfx950",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-o", str(out), src]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert out.stat().st_size > 0
