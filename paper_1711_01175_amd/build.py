"""Build the HIP/C++ library libewdg.so for gfx950 in-tree.

Compiles every source under csrc/ with hipcc and links one shared library
next to this file.  Packed FP32 instructions are disabled for device code.

build_sanitized() compiles the same sources with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only (-Xarch_host before every
sanitizer flag; GPU code is built as usual) and links them with the host
check driver tests/host_check.cpp into _build/san/host_check, a program that
exercises the library's host paths without a GPU.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libewdg.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-I" + CSRC, "-I" + os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))


def _compile(src):
    obj = os.path.join(BUILD, src + ".o")
    # every translation unit is compiled as HIP (host files use the HIP runtime API)
    cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE
    subprocess.run(cmd, check=True)
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, sources()))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH, "-fPIC"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _compile_san(args):
    src, out = args
    cmd = [HIPCC, "-x", "hip", "-c", src, "-o", out, "-O1", "-g", "-fPIC", "-std=c++17",
           "-I" + CSRC, "-I" + os.path.join(ROOT, "include")] + DEVICE + SAN
    subprocess.run(cmd, check=True, stderr=subprocess.DEVNULL)
    return out


def build_sanitized(verbose=False):
    """Host-sanitized build of the library sources and the host check
    driver; returns the path of the executable."""
    san = os.path.join(BUILD, "san")
    os.makedirs(san, exist_ok=True)
    jobs = [(os.path.join(CSRC, f), os.path.join(san, f + ".o")) for f in sources()]
    jobs.append((os.path.join(ROOT, "tests", "host_check.cpp"), os.path.join(san, "host_check.o")))
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile_san, jobs))
    exe = os.path.join(san, "host_check")
    subprocess.run([HIPCC, "-o", exe] + objs + ["--offload-arch=" + ARCH] + SAN, check=True)
    if verbose:
        print("built", exe)
    return exe


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "sanitized":
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
