"""Builds libbst.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2401_01921_amd.build [--force] [-j N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbst.so")
ARCH = "gfx950"

SOURCES = ["structure.cpp", "plan.cpp", "exec.cpp", "lanczos.cpp", "kernels_gemm.hip", "kernels_aux.hip", "kernels_planes.hip",
           "kernels_direct.hip", "kernels_stream.hip", "network.cpp", "kernels_calib.hip",
           "svd.cpp", "kernels_svd.hip"]
HEADERS = ["bst_internal.h", "plan.h", "svd.h", os.path.join("..", "..", "include", "bst.h")]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable"]
# Packed FP32 instructions are kept out of device code on this target.
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _newest_header() -> float:
    return max(os.path.getmtime(os.path.join(CSRC, h)) for h in HEADERS)


def _compile(src: str, force: bool) -> str:
    obj = os.path.join(OBJ, src + ".o")
    srcp = os.path.join(CSRC, src)
    if (not force and os.path.exists(obj) and os.path.getmtime(obj) >= os.path.getmtime(srcp)
            and os.path.getmtime(obj) >= _newest_header()):
        return obj
    cmd = [hipcc()] + COMMON + DEVICE + ["-c", srcp, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc()] + COMMON + ["-x", "hip"] + DEVICE + ["-c", srcp, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{msgs}")
    if msgs.strip():
        sys.stderr.write(msgs + "\n")
    return obj


# Host-code sanitizer build: the C++ sources (tensor structure, plans,
# execution, Lanczos driver, network order) with AddressSanitizer and
# UndefinedBehaviorSanitizer on their host code only, linked with the
# regular kernel objects.  The sanitizer runtime is not linked into the
# library: a process loads it first (LD_PRELOAD of sanitizer_runtime()).
SAN_OBJ = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_OBJ, "libbst_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-g"]


def sanitizer_runtime() -> str:
    import glob
    root = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "lib", "clang")
    hits = sorted(glob.glob(os.path.join(root, "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not hits:
        hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return hits[-1]


def build_sanitized(jobs: int = 8) -> str:
    """Builds SAN_LIB (host sources sanitized, kernels from the regular build)."""
    os.makedirs(SAN_OBJ, exist_ok=True)
    host_src = [s for s in SOURCES if s.endswith(".cpp")]
    kern_objs = [os.path.join(OBJ, s + ".o") for s in SOURCES if s.endswith(".hip")]
    missing = [o for o in kern_objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError("build the library first (kernel objects missing)")

    def comp(src):
        obj = os.path.join(SAN_OBJ, src + ".o")
        srcp = os.path.join(CSRC, src)
        if (os.path.exists(obj) and os.path.getmtime(obj) >= os.path.getmtime(srcp)
                and os.path.getmtime(obj) >= _newest_header()):
            return obj
        cmd = [hipcc()] + COMMON + SAN_FLAGS + ["-x", "hip"] + DEVICE + ["-c", srcp, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized compile failed: {src}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(comp, host_src))
    newest = max(os.path.getmtime(o) for o in objs + kern_objs)
    if os.path.exists(SAN_LIB) and os.path.getmtime(SAN_LIB) >= newest:
        return SAN_LIB
    tmp = SAN_LIB + ".tmp"
    cmd = ([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", tmp] + objs + kern_objs)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed\n" + r.stdout + r.stderr)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def build(force: bool = True, jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=8)
    ap.add_argument("--sanitize", action="store_true",
                    help="also build the host-sanitized library (_build_san/libbst_san.so)")
    a = ap.parse_args()
    build(force=a.force, jobs=a.j, verbose=True)
    if a.sanitize:
        print("built", build_sanitized(jobs=a.j))
