"""Build libmnfpty.so (the HIP kernels and the C ABI) for gfx950 in-tree.

Usage: python -m paper_2608_01746_amd.build  (or call build()).
Every call recompiles all sources.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmnfpty.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the first kernel arguments arrive in SGPRs at wave start (each kernel
    # also carries the loading entry used where the firmware does not preload)
    "-mllvm", "-amdgpu-kernarg-preload-count=16",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = sources()

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    workers = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")), 16)
    with cf.ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


# Host code with AddressSanitizer and UndefinedBehaviorSanitizer.  Device
# code is not compiled (relocatable host-only objects, so no code object is
# referenced): kernels cannot be launched from this build, which serves the
# CPU tests of the host paths (argument validation, planning, tiling).  Load
# it into a process with the ASan runtime preloaded (asan_runtime()).
SANITIZE_FLAGS = [
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
]
SAN_DIR = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_DIR, "libmnfpty_san.so")


def asan_runtime() -> str:
    """Path of the compiler's shared ASan runtime (to preload)."""
    clang = "/opt/rocm/llvm/bin/clang"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the ASan runtime library was not found")
    return path


def _sources_stamp(flags) -> str:
    import hashlib
    h = hashlib.sha256(" ".join(flags).encode())
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def build_host_sanitized() -> str:
    """Build (when the sources changed since the last build) the sanitized
    host-only library and return its path."""
    hipcc = _hipcc()
    flags = ["-fgpu-rdc", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC", *SANITIZE_FLAGS,
             "-Wno-unused-command-line-argument"]
    stamp = _sources_stamp(flags)
    stamp_file = os.path.join(SAN_DIR, "stamp")
    if os.path.exists(SAN_LIB) and os.path.exists(stamp_file) and open(stamp_file).read() == stamp:
        return SAN_LIB
    os.makedirs(SAN_DIR, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(SAN_DIR, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc (sanitized host) failed for {src}:\n{r.stderr}")
        return obj

    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=max(1, min(len(srcs), 8))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = SAN_LIB + ".tmp"
    r = subprocess.run([hipcc, "-fgpu-rdc", "--offload-host-only", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (sanitized host) failed:\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    with open(stamp_file, "w") as fh:
        fh.write(stamp)
    return SAN_LIB


if __name__ == "__main__":
    print(build(verbose=True))
