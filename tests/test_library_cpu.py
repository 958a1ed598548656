"""CPU-side checks of the C-ABI library: it loads and exports every entry point
that include/r1.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2211_14318_amd", "libr1.so")
HDR = os.path.join(ROOT, "include", "r1.h")


def declared():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:r1_status|const char\*)\s+(r1_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("r1_create", "r1_destroy", "r1_envelope", "r1_envelope_stress",
                 "r1_envelope_batched"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libr1.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libr1.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.r1_status_string.restype = ctypes.c_char_p
    assert lib.r1_status_string(0) == b"ok"
    assert lib.r1_status_string(-1) == b"invalid argument"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libr1.so not built")
def test_argument_checks_need_no_gpu():
    """Null handle / null outputs are rejected before any device call."""
    from paper_2211_14318_amd import r1
    L = r1.lib()
    assert L.r1_envelope(None, None, None, 1, 0, None, None, None, None, None) == -1
    assert L.r1_create(None, 0) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libr1.so not built")
def test_check_offsets_schedule():
    """The surrogate check's sample offsets (host logic, r1_surrogate_check_offsets)
    for every odd line length up to R1_MAX_NT: strictly increasing, every offset up
    to 8 (or to the half-length c), the line's end c last, at most 32 of them, and
    beyond 8 each step at most about a third of the previous offset (one more than
    it when that rounds lower); invalid lengths are rejected."""
    from paper_2211_14318_amd import r1
    for n_t in range(3, 2050, 2):
        c = (n_t - 1) // 2
        offs = [int(o) for o in r1.check_offsets(n_t)]
        assert offs[0] == 1 and offs[-1] == c and len(offs) <= 32, n_t
        assert all(b > a for a, b in zip(offs, offs[1:])), n_t
        assert offs[:min(8, c)] == list(range(1, min(8, c) + 1)), n_t
        for a, b in zip(offs[7:-1], offs[8:-1]):
            assert b <= max(a + 1, int(a * 1.3 + 0.5)), (n_t, a, b)
    for bad in (1, 2, 4, 2051):
        with pytest.raises(r1.R1Error):
            r1.check_offsets(bad)


def test_grid_reduced_directions_match_oracle():
    """r1_grid_r11 is host code: the library's reduced direction set (eq. 5.1) equals the
    oracle's, in the same order (16 steps in 2D, 169 in 3D)."""
    from oracle import oracle as O
    from paper_2211_14318_amd import r1
    for dim in (2, 3):
        assert np.array_equal(r1.grid_r11(dim), O.grid_r11(dim))


def test_grid_line_starts_match_brute_force(tmp_path):
    """The grid kernels' line-start decoding (host/device header, built here with the host
    compiler): for random meshes and steps -- zero components, steps longer than the box --
    the decoded starts are exactly the nodes whose predecessor lies outside the box (of the
    lines with at least min_len nodes), each once, with the right line lengths, index step
    and longest line; stepping from a start
    to a later one (mixed-radix add with carry within a slab, by 1 and by 5) agrees with
    decoding."""
    check_grid_lines(build_grid_check(tmp_path / "check"))


def test_fp64_log_exp_accuracy(tmp_path):
    """The FP64 sampling path's own log and exp (csrc/r1_math.hpp, built with the host
    compiler without contraction, so the same operations as on the device): at most
    1.5 units in the last place from the x87 extended-precision logl / expl over the
    positive range, near 1, over [-745, 0] and near 0, and the C library's special values."""
    import subprocess
    exe = tmp_path / "math_check"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-Wall", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "paper_2211_14318_amd", "csrc"),
                           os.path.join(ROOT, "tests", "math_f64_check.cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    worst = {l.split()[1]: float(l.split()[2]) for l in out.splitlines() if l.startswith("max_ulp")}
    assert len(worst) == 7 and out.strip().splitlines()[-1].startswith("ok"), out
    assert max(worst.values()) <= 1.5, worst


def build_grid_check(exe, extra_flags=()):
    import subprocess
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Wno-unknown-pragmas", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "paper_2211_14318_amd", "csrc"),
                           "-I" + os.path.join(ROOT, "include"), *extra_flags,
                           os.path.join(ROOT, "tests", "grid_lines_check.cpp"), "-o", str(exe)])
    return exe


def check_grid_lines(exe):
    """Runs the grid_lines_check harness on 36 random meshes and compares with brute force."""
    import subprocess
    import sys
    sys.path.insert(0, ROOT)
    import bench
    rng = np.random.default_rng(5)
    for trial in range(36):
        dim = 2 if trial % 3 else 3
        dd = dim * dim
        min_len = 1 + trial % 4
        n = [int(v) for v in rng.integers(1, 7 if dim == 2 else 4, size=dd)]
        steps = [[int(v) for v in rng.integers(-3, 4, size=dd)] for _ in range(6)]
        steps = [s for s in steps if any(s)] + [[1] + [0] * (dd - 1), [0] * (dd - 1) + [-7], [1] * dd]
        text = " ".join(map(str, [dim] + n + [len(steps), min_len] + sum(steps, [])))
        out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout.split()
        vals = list(map(int, out))
        pos = 0
        strides = [int(np.prod(n[c + 1:])) for c in range(dd)]
        for s in steps:
            count, longest, ds = vals[pos:pos + 3]
            pos += 3
            got = {}
            for _ in range(count):
                assert vals[pos] not in got
                got[vals[pos]] = vals[pos + 1]
                assert vals[pos + 2] == 1                           # stepping agrees with decoding
                pos += 3
            every = {}
            for I in np.ndindex(*n):
                if all(0 <= I[c] - s[c] < n[c] for c in range(dd)):
                    continue
                L = 0
                while all(0 <= I[c] + L * s[c] < n[c] for c in range(dd)):
                    L += 1
                every[int(np.ravel_multi_index(I, n))] = L
            assert sum(every.values()) == int(np.prod(n))         # the lines partition the mesh
            assert longest == max(every.values())
            assert got == {p: L for p, L in every.items() if L >= min_len}, (n, s, min_len)
            assert count == bench.grid_lines_at_least(n, s, min_len)  # the bench's closed form
            assert ds == sum(s[c] * strides[c] for c in range(dd))
        assert pos == len(vals)


def test_bench_contract_without_gpu(tmp_path):
    """bench.py's host logic: it refuses more than one GPU with a message and a non-zero
    status; the committed HBM traffic figure is reported only while the kernel sources
    hash to the fingerprint it was measured on; the algorithmic byte counts of the
    tangent and grid legs."""
    import subprocess
    import sys
    sys.path.insert(0, ROOT)
    import bench
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""
    assert isinstance(bench.measured_traffic(), int)        # sources unchanged since the counters
    text = open(bench.TRAFFIC_FILE).read()
    stale = tmp_path / "hbm.txt"
    stale.write_text(text.replace("source_fingerprint = ", "source_fingerprint = 0"))
    old = bench.TRAFFIC_FILE
    try:
        bench.TRAFFIC_FILE = str(stale)
        assert bench.measured_traffic() is None
    finally:
        bench.TRAFFIC_FILE = old
    # 2D depth 1, FP32: F (4), beta_n, W, one tree node of 16 B, 16 moduli
    assert bench.tangent_bytes(2, 1, 4) == 4 * (4 + 2) + 16 + 4 * 16
    # a 2D mesh whose lines along component 0 have 5 nodes and no other line has 3
    n = [5, 1, 1, 1]
    steps = [[1, 0, 0, 0], [0, 1, 0, 0]]
    assert bench.grid_line_nodes(n, steps) == 5
    assert bench.grid_bytes(5, 5, 8) == 8 * (5 + 2 * 5)
