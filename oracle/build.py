"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
          "-fno-unsafe-math-optimizations", "-fPIC", "-shared"]


SAN_LIB = os.path.join(HERE, "liboracle_san.so")
# host sanitizers: address (bounds, use after free) and undefined behaviour, stopping at the first report
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def build_sanitized(verbose: bool = False) -> str:
    """The same oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (CPU test
    runs only; load it with gcc's libasan preloaded)."""
    tmp = SAN_LIB + ".tmp"
    cmd = ["gcc"] + [f for f in CFLAGS if f != "-O2"] + SAN_FLAGS + ["-o", tmp, os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc"] + CFLAGS + ["-o", tmp, os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
