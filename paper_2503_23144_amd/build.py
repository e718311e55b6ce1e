"""Build liblrcc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2503_23144_amd.build          # compile every source, link

Objects go to _build/ at the repository root; the library is written next
to this file, where the ctypes binding loads it.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "liblrcc.so")

SOURCES = ["program.cpp", "devmem.hip", "kernels.hip", "gemm.hip", "runtime.hip", "integrals.hip", "solver.hip", "fnspp.hip",
           "abi.hip", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall", "-Wno-unused-result",
         # no packed FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + SRC]


def _compile(src: str) -> str:
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(SRC, src), "-o", out]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + [f for f in FLAGS if f not in ("--offload-arch=gfx950",)] + ["-x", "c++", "-c",
                                                                                    os.path.join(SRC, src), "-o", out]
        cmd = [c for c in cmd if c not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    return out


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(SRC, s))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# Host code under AddressSanitizer and UndefinedBehaviorSanitizer: every
# source compiled as usual for gfx950, the sanitizer flags on the host pass
# only (device code is not instrumented).  It serves host-side checks -- the
# program transforms, the planners, argument checks, the workspace estimate;
# load it with the clang ASan runtime preloaded.
SAN_DIR = os.path.join(OBJ, "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "liblrcc.so")
SAN_FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall", "-Wno-unused-result",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-I" + os.path.join(ROOT, "include"), "-I" + SRC]


def asan_runtime() -> str:
    """Path of the clang ASan runtime that a sanitized library needs preloaded."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang ASan runtime not found under /opt/rocm/llvm")
    return hits[-1]


def _compile_sanitized(src: str) -> str:
    out = os.path.join(SAN_DIR, os.path.splitext(os.path.basename(src))[0] + ".o")
    flags = SAN_FLAGS
    if src.endswith(".cpp"):  # host C++ (host test drivers include the HIP headers)
        flags = [f for f in SAN_FLAGS if f not in ("--offload-arch=gfx950", "-Xclang", "-target-feature",
                                                   "-packed-fp32-ops")]
        flags += ["-x", "c++"] if src.endswith("program.cpp") else ["-x", "hip", "--cuda-host-only"]
    cmd = [HIPCC] + flags + ["-c", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build_sanitized(extra_sources=(), verbose: bool = True) -> str:
    """liblrcc.so with sanitized host code at _build/sanitize/liblrcc.so;
    extra_sources (host C++ files) are compiled the same way and linked into
    executables of their own name next to it."""
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = [os.path.join(SRC, s) for s in SOURCES if os.path.exists(os.path.join(SRC, s))]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile_sanitized, srcs + list(extra_sources)))
    lib_objs, extra_objs = objs[:len(srcs)], objs[len(srcs):]
    link = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-L/opt/rocm/lib",
            "-lamdhip64", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", SAN_LIB] + lib_objs + link
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    for src, obj in zip(extra_sources, extra_objs):
        exe = os.path.join(SAN_DIR, os.path.splitext(os.path.basename(src))[0])
        cmd = [HIPCC, "--offload-arch=gfx950", "-o", exe, obj] + lib_objs + link + ["-Xarch_host", "-shared-libasan"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"built {SAN_LIB}")
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        build_sanitized()
    else:
        build()
