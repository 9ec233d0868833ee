"""Build liblbmd.so (the HIP library) in-tree for gfx950.

    python -m paper_0711_2665_amd.build

Multiply-add contraction is off so that the FP64 path rounds each written
operation exactly once; packed FP32 instructions are disabled.
"""
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbmd.so")
SOURCES = ["lbmd_api.hip", "lb_kernels.hip", "md_kernels.hip", "adj_kernels.hip"]
HEADERS = ["lbmd_dev.h", "lbmd_kernels.h", "lbmd_lattice.h"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [hipcc()] + FLAGS + ["-I" + os.path.join(ROOT, "include"), "-o", LIB + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def kernel_source_hash():
    """Short hash of the sources that define the lattice sweep; a counter
    summary taken on other sources no longer describes the kernel."""
    h = hashlib.sha256()
    for f in ("lb_kernels.hip", "lbmd_dev.h", "lbmd_kernels.h", "lbmd_lattice.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "lbmd.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
