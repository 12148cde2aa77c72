"""Build liblw.so (all HIP sources under csrc/) for gfx950 with hipcc, in-tree.

Usage: python -m paper_2206_03015_amd.build  (or build() from Python).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblw.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: no v_pk_{add,mul,fma}_f32 anywhere in this library.
# -munsafe-fp-atomics: float/double atomicAdd map to the hardware global atomics.
# -ffp-contract=on: fuse only inside one expression (arrival times use explicit fma()).
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer (the device code is built as usual).
# A process that loads such a build needs the compiler's ASan runtime preloaded.
SAN_FLAGS = [f for s in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                         "-fno-omit-frame-pointer", "-g") for f in ("-Xarch_host", s)]


def _compile(src: str, build_dir: str = BUILD_DIR, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-I", INCLUDE, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    """Compile every csrc/*.hip and link liblw.so next to this file (or at ``out``).  Always
    rebuilds.  ``sanitize`` builds the host code with ASan + UBSan into a separate object folder;
    load such a library with ``LW_LIBRARY=<path>`` and the runtime from ``asan_runtime()``
    preloaded."""
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        raise RuntimeError("hipcc not found")
    build_dir = os.path.join(BUILD_DIR, "san") if sanitize else BUILD_DIR
    extra = SAN_FLAGS if sanitize else []
    lib = out or LIB
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir, extra), srcs))
    tmp = lib + ".tmp"
    link_extra = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"] \
        if sanitize else []
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *link_extra, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", LIB)
    return LIB


def asan_runtime() -> str:
    """The ASan shared runtime of the compiler behind hipcc (to preload for a sanitized build)."""
    r = subprocess.run([os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the ASan runtime of hipcc's compiler was not found")
    return path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
