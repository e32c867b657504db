"""Build libqdcb.so (HIP kernels + C-ABI runtime) for gfx950 with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqdcb.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # no packed-FP32 instruction selection (device code)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_sanitized(verbose: bool = False) -> str:
    """CPU check build: the library's host code with AddressSanitizer and
    UndefinedBehaviorSanitizer (device code as usual; the sanitizers are
    passed to the host compilation only), linked into sanitize_check, a
    driver of the entry points that need no device.  Returns its path."""
    out = os.path.join(HERE, "_build_san")
    os.makedirs(out, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + san

    def comp(src):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        r = subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        return obj

    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin")
    clang = os.path.normpath(clang)
    drv_o = os.path.join(out, "sanitize_check.o")
    exe = os.path.join(out, "sanitize_check")
    for cmd in ([os.path.join(clang, "clang"), "-O1", "-g", "-fsanitize=address,undefined",
                 "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-c",
                 os.path.join(HERE, "sanitize_check.c"), "-o", drv_o],
                [os.path.join(clang, "clang++"), "-fsanitize=address,undefined",
                 "-fno-gpu-sanitize", drv_o, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                 "-Wl,-rpath,/opt/rocm/lib", "-o", exe]):
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized build failed:\n{' '.join(cmd)}\n{r.stderr}")
    if verbose:
        print("built", exe)
    return exe


if __name__ == "__main__":
    build(verbose=True)
