"""Build libpt.so (HIP kernels for gfx950 + C-ABI host code) in the package dir."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["kernels.hip", "probe.hip", "capi.hip", "bvh_build.cpp"]
# the vendor library's radix sort behind a C entry point (the sort's yardstick in the benchmark)
SORTREF_LIB = os.path.join(HERE, "libptsortref.so")
SORTREF_SOURCES = ["sort_reference.hip"]

# -ffp-contract=off: the ray chain is binary32 without FMA contraction (host and device).
# -packed-fp32-ops off: no packed FP32 instructions are generated.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-pthread"]


SAN_LIB = os.path.join(HERE, "libpt_san.so")
# host sanitizers for the CPU tests of the host code (scene build, BVH, C-ABI checks, batch
# bookkeeping): address and undefined behaviour on the host side of every source only
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-shared-libsan"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compiles libpt.so; with sanitize, libpt_san.so with host-side ASan and UBSan (load it with
    the compiler's ASan runtime preloaded; for CPU runs of the host code)."""
    out = SAN_LIB if sanitize else LIB
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + SAN_HOST if sanitize else FLAGS
    return _compile(out, flags, SOURCES, verbose)


def build_sortref(verbose: bool = False) -> str:
    """Compiles libptsortref.so (pt_sortref.h)."""
    return _compile(SORTREF_LIB, FLAGS, SORTREF_SOURCES, verbose)


def _compile(out, flags, sources, verbose):
    tmp = out + ".tmp"
    cmd = [HIPCC] + flags + ["-o", tmp] + [os.path.join(CSRC, s) for s in sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose and r.stderr:
        # the host pass does not know the packed-fp32 target feature; that warning is expected
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_sortref(verbose=True))
