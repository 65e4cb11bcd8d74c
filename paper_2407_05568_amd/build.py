"""Build the gfx950 HIP library libesvdw.so in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libesvdw.so")
SOURCES = ["api.hip", "rhs.hip", "mesh.hip", "mlp.hip", "batch.hip"]
ARCH = os.environ.get("ESVDW_ARCH", "gfx950")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose=False):
    """Compile every .hip source for the target architecture and link the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include"),
           "-o", tmp] + sources()
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
