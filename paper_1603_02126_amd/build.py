"""Build the HIP library libepic.so for gfx950 in-tree.

    python -m paper_1603_02126_amd.build        (or __graft_entry__.build())

Every HIP source is compiled with hipcc for gfx950 only; packed-FP32 VALU
instructions are disabled in device code (plain scalar FP32 arithmetic).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libepic.so")

SOURCES = ["epic_api.hip", "k_image.hip", "k_adjoint.hip", "k_solve.hip", "k_dft.hip", "k_batch.hip", "k_fused.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Wall",
        "-Wno-unused-function",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-I", CSRC,
    ]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *common_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libepic.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


ASAN_CHECK = os.path.join(ROOT, "tests", "host_asan", "epic_asan_check.cpp")


def build_asan_check(out_dir: str, device: bool = True, verbose: bool = False) -> str:
    """Build the host-side AddressSanitizer + UndefinedBehaviorSanitizer check
    (tests/host_asan/epic_asan_check.cpp) against freshly compiled library
    objects.  Only the host side of every source is instrumented; device code
    is compiled as usual (device=False compiles the host side alone, for
    machines without a GPU).  Returns the executable's path."""
    os.makedirs(out_dir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    mode = [] if device else ["--offload-host-only"]

    def comp(src):
        obj = os.path.join(out_dir, os.path.splitext(os.path.basename(src))[0] + ".o")
        cmd = [hipcc(), *common_flags(), *mode, *san, "-O1", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [ASAN_CHECK]
    with ThreadPoolExecutor(len(srcs)) as ex:
        objs = list(ex.map(comp, srcs))
    exe = os.path.join(out_dir, "epic_asan_check")
    # the sanitizer runtimes are linked by the host compiler on a line of its own
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    rocm = os.path.realpath(os.path.join(os.path.dirname(os.path.realpath(hipcc())), ".."))
    cmd = [clang, "-fsanitize=address,undefined", *objs, "-o", exe, "-L", os.path.join(rocm, "lib"),
           "-Wl,-rpath," + os.path.join(rocm, "lib"), "-lamdhip64"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    return exe


if __name__ == "__main__":
    if "--asan-check" in sys.argv:
        out = sys.argv[sys.argv.index("--asan-check") + 1]
        print(build_asan_check(out, device="--host-only" not in sys.argv, verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
