"""Build the vkmg HIP library in-tree for gfx950.

    python -m paper_2401_06277_amd.build          # or build() from Python

Compiles the HIP sources with hipcc (device code for gfx950 only, packed
FP32 instructions disabled) and the pure host setup with g++, and links
``paper_2401_06277_amd/libvkmg.so``.  Always rebuilds.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libvkmg.so")

HIP_SOURCES = ["kernels.hip", "api.hip"]
HOST_SOURCES = ["host_setup.cpp"]
GEN_DIR = os.path.join(BUILD, "gen")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Wno-unused-function", "-Wno-unknown-pragmas",
    # no packed FP32 VALU instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I" + GEN_DIR,
]
# machine scheduling that keeps memory clauses together: no spills in the FP64
# residual kernel at its 128-register budget (same arithmetic; FP64 V-cycle at
# 1024^2 about 1 % faster than under the default strategy)
MEMORY_CLAUSE = ["-mllvm", "-amdgpu-sched-strategy=max-memory-clause"]
# (object name, source, extra flags): kernels.hip is compiled as two units, the
# FP64 launchers and everything not tied to a precision under MEMORY_CLAUSE,
# the FP32 launchers under the default strategy (FP32 V-cycle about 2 % faster);
# the same arithmetic either way
HIP_UNITS = [
    ("kernels64", "kernels.hip", ["-DVKMG_KERNEL_UNIT=64", *MEMORY_CLAUSE]),
    ("kernels32", "kernels.hip", ["-DVKMG_KERNEL_UNIT=32"]),
    ("api", "api.hip", MEMORY_CLAUSE),
]
GXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    if verbose and (res.stdout or res.stderr):
        sys.stdout.write(res.stdout + res.stderr)


def generate_headers(verbose: bool = False) -> None:
    """Compile and run the generator of the interior-operator constants."""
    os.makedirs(GEN_DIR, exist_ok=True)
    exe = os.path.join(BUILD, "gen_interior_blocks")
    _run(["g++", *GXX_FLAGS, os.path.join(CSRC, "gen_interior_blocks.cpp"),
          os.path.join(CSRC, "host_setup.cpp"), "-o", exe], verbose)
    res = subprocess.run([exe], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"gen_interior_blocks failed with status {res.returncode}")
    out = os.path.join(GEN_DIR, "interior_blocks.h")
    with open(out + ".tmp", "w") as f:
        f.write(res.stdout)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False, extra_flags=None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    generate_headers(verbose)
    hipcc = _hipcc()
    objs = []
    for name, src, unit_flags in HIP_UNITS:
        obj = os.path.join(BUILD, name + ".o")
        _run([hipcc, *HIPCC_FLAGS, *unit_flags, *(extra_flags or []), "-c",
              os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["g++", *GXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


def _llvm_bin(name: str) -> str:
    for cand in (os.path.join("/opt/rocm/llvm/bin", name), shutil.which(name)):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError(f"{name} not found (ROCm's LLVM is required for the sanitizer build)")


def asan_runtime() -> str:
    """Path of the shared AddressSanitizer runtime of ROCm's clang (to be
    preloaded into a process that loads the sanitized library)."""
    res = subprocess.run([_llvm_bin("clang++"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode != 0 or not os.path.exists(path):
        raise RuntimeError("clang's shared ASan runtime not found")
    return path


def build_sanitized(verbose: bool = False) -> str:
    """CPU-only build of the library with AddressSanitizer and
    UndefinedBehaviorSanitizer on the host code (the setup, the argument
    validation and every host path of the C ABI); device code unchanged.
    Writes _build/sanitize/libvkmg_sanitized.so, which a process loads with
    the runtime of asan_runtime() preloaded.  Never used on a GPU."""
    out_dir = os.path.join(BUILD, "sanitize")
    os.makedirs(out_dir, exist_ok=True)
    generate_headers(verbose)
    hipcc = _hipcc()
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        _run([hipcc, *HIPCC_FLAGS, *host_san, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    cxx = _llvm_bin("clang++")
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        _run([cxx, *GXX_FLAGS, *san, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    lib = os.path.join(out_dir, "libvkmg_sanitized.so")
    _run([cxx, "-shared", "-fPIC", *san, "-shared-libsan", "-o", lib, *objs,
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], verbose)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
