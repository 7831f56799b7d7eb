"""Build libpe.so (the HIP library behind include/pe.h) in-tree for gfx950 with hipcc.

Packed FP32 instructions are disabled for all device code
(-target-feature -packed-fp32-ops); hipcc's host pass warns that it does not
know the feature, which is harmless.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpe.so")
SOURCES = ["pe_kernels.hip", "pe_loglike.hip", "pe_api.hip", "pe_server.hip", "pe_tiles.hip", "pe_relbin.hip"]
ARCH = os.environ.get("PE_OFFLOAD_ARCH", "gfx950")


def build(verbose=False, save_temps_dir=None):
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-Wall", "-Wno-unused-function", "-Wno-unused-result"]
    if save_temps_dir:
        os.makedirs(save_temps_dir, exist_ok=True)
        cmd += [f"-save-temps={'obj'}"]
    cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    cwd = save_temps_dir or HERE
    subprocess.check_call(cmd, cwd=cwd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
