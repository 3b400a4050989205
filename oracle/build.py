"""Compile the FP64 CPU oracle (test infrastructure) with gcc.

Usage: python oracle/build.py              -> oracle/liboracle.so
       python oracle/build.py --sanitize   -> oracle/liboracle_san.so, built
           with AddressSanitizer and UndefinedBehaviorSanitizer (host code
           only).  The oracle package loads it instead of liboracle.so when
           ORACLE_SANITIZED=1; the sanitizer runtime must then be preloaded:
           LD_PRELOAD=$(gcc -print-file-name=libasan.so) ASAN_OPTIONS=detect_leaks=0
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rbm_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")
OUT_SAN = os.path.join(HERE, "liboracle_san.so")
SANITIZE = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    # -O2, no fast-math: strict IEEE FP64 so the oracle's rounding is the
    # plain C rounding of each written operation; -ffp-contract=off keeps
    # a*b+c as two roundings.  -fopenmp: parallel loops over particles (the
    # per-particle arithmetic does not depend on the thread count).
    out = OUT_SAN if sanitize else OUT
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra"]
    if sanitize:
        cmd += SANITIZE
    cmd += ["-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv, sanitize="--sanitize" in sys.argv))
