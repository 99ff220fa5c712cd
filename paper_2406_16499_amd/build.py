"""Build liblsq.so (HIP, gfx950) in-tree.

    python -m paper_2406_16499_amd.build        # or build() from Python

Every call compiles from source: one hipcc invocation per translation unit
(in parallel) and one link step.  Packed FP32 instructions (v_pk_*_f32) are
disabled for the device code: some of their forms have given wrong results on
this hardware without any error, so the compiler must not form them.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblsq.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["qr.hip", "vec.hip", "blas.hip", "gmres.hip", "selector.hip", "batch.hip", "api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
              shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


COMMON = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-munsafe-fp-atomics"]


POISON_LIB = os.path.join(HERE, "liblsq_poison.so")


def _compile(src: str, variant: str = "") -> str:
    out_dir = os.path.join(BUILD_DIR, variant) if variant else BUILD_DIR
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    extra = ["-DLSQ_POISON_LDS"] if variant == "poison" else []
    cmd = [hipcc(), *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{out}")
    if out.strip():
        sys.stderr.write(out + "\n")
    return obj


def build(verbose: bool = False, variant: str = "") -> str:
    """liblsq.so, or with variant "poison" the debug library liblsq_poison.so
    whose kernels fill their LDS with NaN patterns before first use."""
    lib = POISON_LIB if variant == "poison" else LIB
    os.makedirs(os.path.join(BUILD_DIR, variant) if variant else BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, variant), SOURCES))
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking {os.path.basename(lib)} failed:\n" + r.stdout)
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


SANITIZERS = {"address": "asan", "thread": "tsan"}


def build_sanitized(kind: str = "address", verbose: bool = False) -> str:
    """The library's sources and the host driver csrc/sanitize_driver.cpp built
    into one executable with a host-code sanitizer (AddressSanitizer or
    ThreadSanitizer): every -fsanitize flag applies to the host compilation
    only (-Xarch_host); the device code is built as for liblsq.so.  Returns the
    executable's path (lsq_<asan|tsan>_driver beside liblsq.so)."""
    tag = SANITIZERS[kind]
    out_dir = os.path.join(BUILD_DIR, tag)
    os.makedirs(out_dir, exist_ok=True)
    host = ["-Xarch_host", f"-fsanitize={kind}", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    flags = [f if f != "-O3" else "-O1" for f in COMMON] + host

    def comp(src):
        obj = os.path.join(out_dir, os.path.splitext(os.path.basename(src))[0] + ".o")
        extra = ["-x", "hip"] if src.endswith(".cpp") else []
        r = subprocess.run([hipcc(), *flags, *extra, "-c", src, "-o", obj], stdout=subprocess.PIPE,
                           stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} ({kind}) failed:\n{r.stdout}")
        return obj

    srcs = [os.path.join(CSRC, f) for f in SOURCES] + [os.path.join(CSRC, "sanitize_driver.cpp")]
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(comp, srcs))
    exe = os.path.join(HERE, f"lsq_{tag}_driver")
    r = subprocess.run([hipcc(), f"--offload-arch={ARCH}", *host, "-o", exe, *objs],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking the {kind} driver failed:\n" + r.stdout)
    if verbose:
        print("built", exe)
    return exe


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "sanitize":
        build_sanitized(sys.argv[2], verbose=True)
    elif len(sys.argv) > 1 and sys.argv[1] == "poison":
        build(verbose=True, variant="poison")
    else:
        build(verbose=True)
