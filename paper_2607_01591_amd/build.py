"""Build libmoc.so in-tree with hipcc for gfx950.

Usage: ``python -m paper_2607_01591_amd.build`` (or ``build()`` from Python). Sources are
compiled in parallel into ``_build/`` objects and linked into
``paper_2607_01591_amd/libmoc.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmoc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["moc_setup.cpp", "moc_pack.cpp", "moc_api.cpp", "moc_kernels.hip", "moc_cmfd.hip", "dg_api.cpp",
           "dg_kernels.hip", "dfem_api.cpp", "dfem_kernels.hip", "hfem_api.cpp", "hfem_kernels.hip", "cnn_kernels.hip"]

# Packed FP32 instructions are disabled for all device code: hipcc would otherwise form
# them from ordinary float arithmetic.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + INCLUDE, "-I" + CSRC]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + HIP_FLAGS + ["-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + HIP_FLAGS + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# Host sanitizers: AddressSanitizer and UndefinedBehaviorSanitizer on the host C++ of the
# setup (mesh, tracking, laydown, links, volumes, packing, coarse mesh, DFEM-SN schedule,
# HFEM set-up). Only host compilation is instrumented (each flag after -Xarch_host); the
# device objects are the regular ones. The library references the sanitizer runtime, which
# the process must preload (clang's libclang_rt.asan, see sanitizer_runtime()).
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
HOST_SOURCES = [s for s in SOURCES if s.endswith(".cpp")]


def sanitizer_runtime() -> str:
    """Path of clang's AddressSanitizer runtime matching hipcc's host compiler."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        import glob
        hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
        if not hits:
            raise RuntimeError("clang AddressSanitizer runtime not found")
        path = hits[-1]
    return path


def build_sanitized(out_dir: str) -> str:
    """libmoc with the host C++ instrumented; device objects from a regular build()."""
    os.makedirs(out_dir, exist_ok=True)
    if not all(os.path.exists(os.path.join(BUILD, s + ".o")) for s in SOURCES if s not in HOST_SOURCES):
        build(verbose=False)

    def comp(src):
        obj = os.path.join(out_dir, src + ".o")
        cmd = [HIPCC, "-x", "hip"] + HIP_FLAGS + SAN_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        objs = list(ex.map(comp, HOST_SOURCES))
    objs += [os.path.join(BUILD, s + ".o") for s in SOURCES if s not in HOST_SOURCES]
    out = os.path.join(out_dir, "libmoc_san.so")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
