"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code.

* The FP64 oracle (plain C) with a driver that calls every exported routine
  on small inputs (tests/helpers/oracle_sanitize_main.c).
* The library's host runtime (input validation, workspace layout, size
  queries, argument checks) with a driver that calls the entry points that
  need no GPU (tests/helpers/host_sanitize_main.c).  Only the host side is
  instrumented: every sanitizer flag is given to the host compilation alone.

Both run on the CPU; a sanitizer report or a failed check fails the test."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HELP = os.path.join(ROOT, "tests", "helpers")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    p = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tempfile.mkdtemp(prefix="orc_san_")
    exe = os.path.join(d, "orc_san")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", *SAN, "-o", exe,
                    os.path.join(HELP, "oracle_sanitize_main.c"),
                    os.path.join(ROOT, "oracle", "ara_oracle.c"), "-lm"], check=True)
    assert "all checks held" in _run(exe)


def test_host_runtime_under_sanitizers():
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_1501_06326_amd import build as B
    d = tempfile.mkdtemp(prefix="host_san_")
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    objs = []
    procs = []
    for src in B.SOURCES:
        obj = os.path.join(d, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen(
            [hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "-pthread", f"--offload-arch={B.ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san,
             "-I", os.path.join(ROOT, "include"), "-I", B.CSRC, "-c",
             os.path.join(B.CSRC, src), "-o", obj],
            stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err.decode()[-3000:]
    exe = os.path.join(d, "host_san")
    subprocess.run([hipcc, "-g", *host_san, f"--offload-arch={B.ARCH}", "-pthread",
                    "-I", os.path.join(ROOT, "include"), "-x", "c",
                    os.path.join(HELP, "host_sanitize_main.c"), "-x", "none", *objs, "-o", exe],
                   check=True, stdout=subprocess.DEVNULL)
    assert "all checks held" in _run(exe)
