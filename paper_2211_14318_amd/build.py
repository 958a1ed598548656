"""Builds libr1.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2211_14318_amd.build [--sanitize]   (or __graft_entry__.build())
Every .hip / .cpp under csrc/ is compiled as HIP for gfx950 in parallel and
linked into paper_2211_14318_amd/libr1.so.

--sanitize builds libr1_san.so instead, the configuration the CPU tests check
host code with: the host-only .cpp files (argument checks, planning, caches,
the C-ABI entry points) compiled with AddressSanitizer and
UndefinedBehaviorSanitizer on the host pass, the .hip files (kernels and
their launchers) reused from libr1.so's objects, linked by the ROCm clang
against its shared sanitizer runtime.  Nothing sanitized runs on the GPU.
Loading it needs that runtime preloaded (LD_PRELOAD=san_runtime()), and
R1_LIB_SANITIZE=1 makes r1.py load it.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libr1.so")
LIB_SAN = os.path.join(PKG, "libr1_san.so")
BUILD_SAN = os.path.join(PKG, "_build_san")
ARCH = "gfx950"
# the sanitized build: sanitizers on the host pass only, each flag behind -Xarch_host
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN_LINK = ["-fsanitize=address,undefined", "-shared-libsan"]
SAN_RUNTIME = os.path.join(os.path.dirname(os.path.realpath(CLANG)), "..", "lib", "clang")

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Wall", "-Wno-unused-result",
]


def _compile(src, san=False):
    obj = os.path.join(BUILD_SAN if san else BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", "-x", "hip", "-c", src, "-o", obj] + CFLAGS + (HOST_SAN if san else [])
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature: drop that warning
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s\n%s" % (src, err))
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def san_runtime():
    """The ROCm clang's shared AddressSanitizer runtime (it carries the UBSan handlers too)."""
    found = sorted(glob.glob(os.path.join(SAN_RUNTIME, "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not found:
        raise RuntimeError("no libclang_rt.asan-x86_64.so under " + SAN_RUNTIME)
    return os.path.realpath(found[-1])


def _fresh(obj):
    """obj is newer than every source and header of the library."""
    if not os.path.exists(obj):
        return False
    deps = glob.glob(os.path.join(CSRC, "*")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    return os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in deps)


def build_sanitized(jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(BUILD_SAN, exist_ok=True)
    hip = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    host = sorted(glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = [f.result() for f in
                [ex.submit(lambda s: os.path.join(BUILD, os.path.basename(s) + ".o")
                           if _fresh(os.path.join(BUILD, os.path.basename(s) + ".o")) else _compile(s), s)
                 for s in hip] + [ex.submit(_compile, s, True) for s in host]]
    tmp = LIB_SAN + ".tmp"
    cmd = [CLANG, "-shared", "-fPIC", "-o", tmp] + SAN_LINK + objs + [
        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stderr)
    os.replace(tmp, LIB_SAN)
    return LIB_SAN


def build(jobs=None, sanitize=False):
    if sanitize:
        return build_sanitized(jobs)
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(sanitize="--sanitize" in sys.argv[1:]))
