"""CPU: host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Two programs are built and run here (no GPU needed):
  * the C oracle with tests/sanitize/oracle_driver.c (gcc), every entry
    point on small, ragged and degenerate inputs;
  * libcmif's host code (plan construction and validation, workspace
    sizes, plan queries, the corner-error measure) with
    tests/sanitize/plan_driver.cpp: api.cpp and noalloc.hip are compiled
    with host-only sanitizers (-Xarch_host before each -fsanitize=) and
    linked with the library's other objects from the in-tree build.
Any sanitizer report aborts the program (-fno-sanitize-recover=all)."""

import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
           OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd[0], r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fopenmp",
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "cmif_oracle.c"), "-lm", "-o", exe])
    out = _run([exe], env=ENV)
    assert "oracle sanitizer driver ok" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    build = os.path.join(ROOT, "paper_2106_14699_amd", "_build")
    others = [o for o in glob.glob(os.path.join(build, "*.o"))
              if os.path.basename(o) not in ("api.o", "noalloc.o")]
    if not others:
        pytest.skip("the in-tree build (paper_2106_14699_amd/_build) is missing")
    csrc = os.path.join(ROOT, "paper_2106_14699_amd", "csrc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fsanitize=undefined"]
    flags = ["-xhip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
             "-fPIC", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", *san, "-Xarch_host", "-fno-sanitize-recover=all",
             "-Xarch_host", "-fno-omit-frame-pointer", "-I",
             os.path.join(ROOT, "include"), "-I", csrc]
    objs = []
    for src in ("api.cpp", "noalloc.hip"):
        o = str(tmp_path / (src + ".o"))
        _run([HIPCC, *flags, "-c", os.path.join(csrc, src), "-o", o])
        objs.append(o)
    exe = str(tmp_path / "plan_san")
    _run([HIPCC, "--offload-arch=gfx950", "-std=c++17", "-x", "c++", *san,
          "-I", os.path.join(ROOT, "include"),
          os.path.join(ROOT, "tests", "sanitize", "plan_driver.cpp"), "-x",
          "none", *objs, *others, "-o", exe])
    out = _run([exe], env=ENV)
    assert "plan sanitizer driver ok" in out
