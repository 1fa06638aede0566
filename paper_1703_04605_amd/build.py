"""Builds the HIP library librlbm.so (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librlbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def build(verbose=False):
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    host_obj = os.path.join(HERE, "_build", "rlbm_stencil.o")
    dev_obj = os.path.join(HERE, "_build", "rlbm_lib.o")
    mlp_obj = os.path.join(HERE, "_build", "rlbm_mlp.o")
    gen_exe = os.path.join(HERE, "_build", "gen_fixed_stencils")
    gen_hdr = os.path.join(HERE, "_build", "rlbm_fixed_stencils.h")
    cmds = [
        ["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", os.path.join(CSRC, "rlbm_stencil.cpp"), "-o", host_obj],
        # fixed-stencil class code, generated from the library's own table builder
        ["g++", "-O2", "-std=c++17", "-Wall", os.path.join(CSRC, "gen_fixed_stencils.cpp"), host_obj, "-o", gen_exe],
        [gen_exe, gen_hdr],
        [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "rlbm_mlp.hip"), "-o", mlp_obj],
        [HIPCC] + HIP_FLAGS + ["-I", os.path.join(HERE, "_build"), "-c", os.path.join(CSRC, "rlbm_lib.hip"), "-o", dev_obj],
        [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", dev_obj, mlp_obj, host_obj, "-o", LIB + ".tmp"],
    ]
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("build failed: " + " ".join(cmd))
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
