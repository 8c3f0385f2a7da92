"""AddressSanitizer + UndefinedBehaviorSanitizer runs on the CPU: the library's
host sources (sampler, parameter compile, tune cache, error reporting) through
tests/host_san.cpp, and the oracle's C code under a selection of its pins."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1809_06839_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _gcc_lib(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_sources_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_san")
    srcs = [os.path.join(ROOT, "tests", "host_san.cpp")] + [os.path.join(CSRC, f) for f in
                                                             ("sampler.cpp", "params.cpp", "runtime.cpp", "errors.cpp")]
    cmd = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")] + \
        SAN + srcs + ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])


@pytest.mark.skipif(_gcc_lib("libasan.so") is None, reason="gcc's libasan not found")
def test_oracle_pins_under_asan_ubsan():
    pre = ":".join(p for p in (_gcc_lib("libasan.so"), _gcc_lib("libubsan.so")) if p)
    env = dict(os.environ, ORACLE_SANITIZE="1", LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    tests = [os.path.join(ROOT, "tests", t) for t in ("test_oracle_primitives.py", "test_oracle_geometry.py",
                                                      "test_oracle_color.py", "test_oracle_pipelines.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + tests,
                       cwd=ROOT, capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
