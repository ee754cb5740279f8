"""Build librd.so (HIP for gfx950) in-tree: one object per source, compiled in
parallel with hipcc, linked into paper_1309_1720_amd/librd.so."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-x", "hip", "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # every rounding where the source writes it (no implicit FMA contraction)
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (res.stdout + res.stderr).splitlines()
            if "packed-fp32-ops" not in l and l.strip()]
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source and link librd.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 4, 16))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


ASAN_BUILD = os.path.join(PKG, "_build_asan")
ASAN_LIB = os.path.join(ASAN_BUILD, "librd_asan.so")


def _stale(obj: str, src: str) -> bool:
    """Whether `obj` is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(PKG, "..", "include", "rd.h"))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def asan_runtime() -> str:
    """Path of the compiler's AddressSanitizer runtime (to LD_PRELOAD into a
    process that loads the instrumented library)."""
    llvm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    import glob
    hits = sorted(glob.glob(os.path.join(llvm, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("no libclang_rt.asan-x86_64.so under the ROCm LLVM")
    return hits[-1]


def build_asan(verbose: bool = False) -> str:
    """librd_asan.so: the host-side sources (the C ABI's validation, workspace
    layout, planning and launch sequencing in the .cpp files) compiled with
    AddressSanitizer on the HOST only, linked with the regular objects of
    the kernel sources.  For CPU-only checks of the ABI (no kernel is
    launched); the device code is not instrumented."""
    if any(_stale(os.path.join(BUILD, os.path.basename(s) + ".o"), s) for s in sources()):
        build(verbose)  # the regular objects (and librd.so) first
    os.makedirs(ASAN_BUILD, exist_ok=True)
    objs = []
    for src in sources():
        base = os.path.basename(src)
        if src.endswith(".cpp"):
            obj = os.path.join(ASAN_BUILD, base + ".o")
            objs.append(obj)
            if not _stale(obj, src):
                continue
            cmd = [HIPCC, *FLAGS, "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
                   "-g", "-c", src, "-o", obj]
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError(f"hipcc (asan) failed on {src}:\n{res.stdout}{res.stderr}")
        else:
            objs.append(os.path.join(BUILD, base + ".o"))
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
           *objs, "-o", ASAN_LIB]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("asan link failed:\n" + res.stdout + res.stderr)
    return ASAN_LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    if "--asan" in sys.argv:
        print(build_asan(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
