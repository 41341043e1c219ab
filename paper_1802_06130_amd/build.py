"""Build libmdn.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1802_06130_amd.build [--jobs N] [--sanitize address|thread]

--sanitize builds a variant whose host code (argument checks, plans, the serving loop and its
threads, the allocator) carries AddressSanitizer or ThreadSanitizer instrumentation, as
_build/<kind>/libmdn.so; the device code is built as usual. Load it with MDN_LIB set to that path
and the matching clang runtime preloaded (sanitizer_runtime()).
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
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmdn.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are kept out of every code object: the kernels use plain
# scalar float math only.
COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Werror=uninitialized",
]


SANITIZE_FLAGS = {
    # host-only instrumentation: every -fsanitize= sits behind -Xarch_host
    "address": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"],
    "thread": ["-Xarch_host", "-fsanitize=thread", "-g"],
}


def sanitizer_runtime(kind: str) -> str:
    """The clang runtime to preload into an uninstrumented interpreter for a sanitized build."""
    name = {"address": "asan", "thread": "tsan"}[kind]
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt." + name + "-x86_64.so"], capture_output=True,
                       text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        rd = subprocess.run([HIPCC, "-print-resource-dir"], capture_output=True, text=True).stdout.strip()
        path = os.path.join(rd, "lib", "linux", "libclang_rt." + name + "-x86_64.so")
    return path


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, sanitize: str | None = None) -> str:
    extra = SANITIZE_FLAGS[sanitize] if sanitize else []
    build_dir = os.path.join(BUILD, sanitize) if sanitize else BUILD
    lib = os.path.join(build_dir, "libmdn.so") if sanitize else LIB
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    j = None
    if "--jobs" in sys.argv:
        j = int(sys.argv[sys.argv.index("--jobs") + 1])
    san = None
    if "--sanitize" in sys.argv:
        san = sys.argv[sys.argv.index("--sanitize") + 1]
    build(j, verbose=True, sanitize=san)
