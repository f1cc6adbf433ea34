"""Builds the FP64 CPU oracle (test infrastructure) into oracle/liblbm_oracle.so.

`python oracle/build.py --sanitize` builds liblbm_oracle_san.so with AddressSanitizer
and UndefinedBehaviorSanitizer (gcc's runtimes must then be preloaded: LD_PRELOAD of
libasan.so and libubsan.so)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.cpp")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    lib = LIB.replace(".so", "_san.so") if sanitize else LIB
    san = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined"] if sanitize else []
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall"] + san + [SRC, "-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    import sys
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
