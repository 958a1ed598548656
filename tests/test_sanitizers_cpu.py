"""The CPU tier under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
  - the oracle's C entry points, driven by tests/oracle_san_check.c (both dimensions,
    both energies, depth 1 and 2, trees, tangent moduli, degenerate F, hulls with
    inadmissible samples, grids, the relax-then-fix driver, the MLP), built with gcc's
    sanitizers;
  - the uneven batch's work planner (tests/batched_plan_check.cpp) and the grid kernels'
    line-start decoding (tests/grid_lines_check.cpp), both host code of the library's
    own headers, built with g++'s sanitizers;
  - the whole CPU suite again with the sanitized builds of both libraries
    (liboracle_san.so; libr1_san.so, whose host C++ is instrumented) loaded under the
    ROCm clang's shared sanitizer runtime.  Skipped, with the reason, when the process
    environment already preloads a library: that preload is left as it is.
Any sanitizer report ends the instrumented process with a non-zero status.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from tests.test_library_cpu import build_grid_check, check_grid_lines  # noqa: E402

GCC_SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
SAN_ENV = dict(ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
    return r.stdout


def test_oracle_entry_points_under_sanitizers(tmp_path):
    from oracle import oracle as O
    exe = str(tmp_path / "oracle_san_check")
    srcs = [os.path.join(ROOT, "oracle", s) for s in O.SOURCES]
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", *GCC_SAN, "-I" + os.path.join(ROOT, "oracle"),
                           os.path.join(ROOT, "tests", "oracle_san_check.c"), *srcs, "-lm", "-o", exe])
    out = _run([exe], env=dict(os.environ, **SAN_ENV))
    assert out.startswith("ok "), out


def test_batched_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "batched_plan_check")
    subprocess.check_call(["g++", "-std=c++17", "-Wall", "-Wextra", *GCC_SAN,
                           "-I" + os.path.join(ROOT, "paper_2211_14318_amd", "csrc"),
                           os.path.join(ROOT, "tests", "batched_plan_check.cpp"), "-o", exe])
    out = _run([exe], env=dict(os.environ, **SAN_ENV))
    assert out.strip() == "ok 300", out


def test_grid_line_decoding_under_sanitizers(tmp_path):
    check_grid_lines(build_grid_check(tmp_path / "grid_lines_check", GCC_SAN))


def _preload_in_use():
    return bool(os.environ.get("LD_PRELOAD")) or os.path.exists("/etc/ld.so.preload")


@pytest.mark.skipif(_preload_in_use(), reason="a library is already preloaded into this environment; "
                                              "the sanitizer runtime would have to replace it")
def test_cpu_suite_under_sanitizers():
    from oracle import oracle as O
    from paper_2211_14318_amd import build as B
    O.build(force=False, sanitize=True)
    if not os.path.exists(B.LIB_SAN) or (os.path.exists(B.LIB)
                                         and os.path.getmtime(B.LIB_SAN) < os.path.getmtime(B.LIB)):
        B.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=B.san_runtime(), R1_ORACLE_SANITIZE="1", R1_LIB_SANITIZE="1", **SAN_ENV)
    # the instrumented builds are the ones loaded
    probe = ("from oracle import oracle as O; from paper_2211_14318_amd import r1; O.lib(); r1.lib(); "
             "m = open('/proc/self/maps').read(); print('liboracle_san.so' in m, 'libr1_san.so' in m)")
    assert _run([sys.executable, "-c", probe], env=env, cwd=ROOT).split() == ["True", "True"]
    out = _run([sys.executable, "-m", "pytest", "tests", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                "--ignore=" + os.path.join("tests", "test_sanitizers_cpu.py")], env=env, cwd=ROOT, timeout=1200)
    assert " passed" in out and " failed" not in out, out[-2000:]
