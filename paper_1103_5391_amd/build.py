"""Builds libdmrgtst.so (the HIP library behind include/dmrgtst.h) for gfx950 with hipcc.

    python -m paper_1103_5391_amd.build            (or build() from Python)
    python -m paper_1103_5391_amd.build --sanitize (host code with AddressSanitizer and
                                                    UndefinedBehaviorSanitizer, see below)

Every source is compiled to its own object under _build/ (in parallel), then linked.

The sanitized variant, libdmrgtst_san.so, rebuilds the host-only sources (the C ABI and the
planner) with -fsanitize=address,undefined for the host pass only (the device code is the normal
objects; GPU sanitizers are not used).  Load it with the clang ASan runtime preloaded:
    LD_PRELOAD=<clang>/lib/linux/libclang_rt.asan-x86_64.so DMRG_LIB=<path> python ...
(asan_runtime() gives the path).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdmrgtst.so")
LIB_SAN = os.path.join(HERE, "_build", "libdmrgtst_san.so")
OBJDIR = os.path.join(HERE, "_build")
HOST_SOURCES = ["csrc/api.cpp", "csrc/plan.cpp", "csrc/tune_cache.cpp"]
DEVICE_SOURCES = ["csrc/gemm.hip", "csrc/gemm_lds.hip", "csrc/gemm_x.hip", "csrc/krylov.hip",
                  "csrc/density.hip", "csrc/wft.hip", "csrc/noalloc.hip", "csrc/gemm_k.hip"]
SOURCES = HOST_SOURCES + DEVICE_SOURCES
ARCH = os.environ.get("DMRG_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 vector ops are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
# host pass only: each -fsanitize= directly after -Xarch_host
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all",
             "-g"]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


def _obj(src: str, tag: str) -> str:
    base = os.path.splitext(os.path.basename(src))[0]
    return os.path.join(OBJDIR, f"{base}{tag}.o")


def _compile(src: str, tag: str, extra, verbose: bool) -> str:
    obj = _obj(src, tag)
    _run([_hipcc(), *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(HERE, src), "-o", obj], verbose)
    return obj


def _link(objs, out: str, extra, verbose: bool) -> str:
    tmp = out + ".tmp"
    _run([_hipcc(), *FLAGS, *extra, "-shared", *objs, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compiles every source (always) and links libdmrgtst.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, "", [], verbose), SOURCES))
    return _link(objs, LIB, [], verbose)


def build_sanitized(verbose: bool = False, jobs: int = 8) -> str:
    """libdmrgtst_san.so: host sources with ASan/UBSan, device sources as in build() (compiled
    if their objects are missing)."""
    os.makedirs(OBJDIR, exist_ok=True)

    def one(src):
        if src in HOST_SOURCES:
            return _compile(src, "_san", SAN_FLAGS, verbose)
        obj = _obj(src, "")
        return obj if os.path.exists(obj) else _compile(src, "", [], verbose)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, SOURCES))
    return _link(objs, LIB_SAN, SAN_FLAGS, verbose)


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime the sanitized library links against."""
    llvm = os.path.dirname(os.path.dirname(os.path.realpath(_hipcc())))
    hits = sorted(glob.glob(os.path.join("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")) +
                  glob.glob(os.path.join(llvm, "llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("clang ASan runtime not found")
    return hits[-1]


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
