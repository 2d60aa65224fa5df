"""Build liblsx.so (HIP/C++ for gfx950) in-tree with hipcc.

    python -m paper_2103_14897_amd.build
    python -m paper_2103_14897_amd.build --host-asan   # also _build/liblsx_host_asan.so

--host-asan builds a second library whose host code (lsx_host.cpp) is instrumented with
AddressSanitizer; the device code is the same as the product's and is not instrumented.  It
is for the CPU tests of the host code (see README.md), loaded through LSX_LIB with the
sanitizer runtime preloaded; it is never the product library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "liblsx.so")

ARCH = os.environ.get("LSX_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC, "-Wall", "-Wno-unused-function",
          # packed FP32 VALU forms are kept out of every code object
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = ["lsx_host.cpp", "lsx_kernels.hip", "lsx_sample.hip"]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_host_asan(verbose=False):
    """_build/liblsx_host_asan.so: the product's device objects with an AddressSanitizer build
    of the host code (sanitizer flags on the host side only)."""
    build(verbose)
    obj = os.path.join(BUILD, "lsx_host_asan.o")
    # host-side only: each sanitizer flag follows -Xarch_host
    san = ["-Xarch_host", "-fsanitize=address"]
    flags = [f for f in COMMON if f != "-O3"] + ["-O1", "-g", *san, "-Xarch_host", "-fno-omit-frame-pointer"]
    r = subprocess.run(["hipcc", *flags, "-c", os.path.join(CSRC, "lsx_host.cpp"), "-o", obj],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for lsx_host.cpp (sanitized):\n{r.stderr}")
    out = os.path.join(BUILD, "liblsx_host_asan.so")
    objs = [obj] + [os.path.join(BUILD, s + ".o") for s in SOURCES if s != "lsx_host.cpp"]
    r = subprocess.run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *san, *objs, "-o", out],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    if "--host-asan" in sys.argv[1:]:
        build_host_asan(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
