"""Host code under the address and undefined-behaviour sanitizers (no GPU).

The library's host geometry (pair list, cube domains, epsilon-box run search
and intersections; csrc/host_geometry.h) and the C oracle are built with
g++ / gcc -fsanitize=address,undefined and driven by small harnesses
(tests/host/); any sanitizer report or failed check fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_geometry_under_sanitizers(tmp_path):
    exe = str(tmp_path / "geom")
    rc, out = _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2208_06097_amd", "csrc"),
                    os.path.join(HERE, "host", "sanitize_geometry.cpp"), "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe], env=ENV, timeout=600)
    print(out)
    assert rc == 0 and "0 failures" in out, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "orc")
    rc, out = _run(["gcc", "-std=c11", *SAN, "-fopenmp", os.path.join(ROOT, "oracle", "sea_oracle.c"),
                    os.path.join(HERE, "host", "sanitize_oracle.c"), "-o", exe, "-lm"])
    assert rc == 0, out
    rc, out = _run([exe], env=ENV, timeout=600)
    print(out)
    assert rc == 0 and "0 failures" in out, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
