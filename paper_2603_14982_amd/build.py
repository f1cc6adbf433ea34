"""Builds the HIP library (gfx950) in-tree: paper_2603_14982_amd/liblbmx.so.

`python build.py --sanitize` builds liblbmx_san.so instead: the host code (runtime,
launchers) with AddressSanitizer and UndefinedBehaviorSanitizer, the GPU code as
usual. Load it with clang's ASan runtime preloaded (LD_PRELOAD of
libclang_rt.asan-x86_64.so) for CPU-side runs of the host code."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblbmx.so")

SOURCES = ["stream_collide.hip", "adjoint.hip", "transfer.hip", "hierarchy.hip", "io.hip", "scalar.hip",
           "runtime.cpp"]
ARCH = os.environ.get("LBMX_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay off: some of their forms are unreliable on this part
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC, "-Wall"]


SAN_FLAGS = ["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
             "-fsanitize=undefined", "-shared-libsan"]


def _compile(src, verbose, sanitize=False):
    obj = os.path.join(BUILD, src + (".san.o" if sanitize else ".o"))
    cmd = ["hipcc"] + FLAGS + (SAN_FLAGS if sanitize else []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, sanitize), SOURCES))
    lib = LIB.replace(".so", "_san.so") if sanitize else LIB
    extra = ["-Xarch_host", "-fsanitize=address,undefined", "-shared-libsan"] if sanitize else []
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC"] + extra + objs + ["-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    import sys
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
