"""Builds liblbmtree.so (HIP for gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbmtree.so")
SOURCES = ["lbm_kernels.hip", "lbm_amr_kernels.hip", "lbm_persist.hip", "lbm_runtime.cpp", "lbm_levels.cpp",
           "lbm_geometry.cpp", "lbm_extra.cpp", "lbm_tune.cpp", "lbm_inflow.cpp", "lbm_inflow.hip",
           "lbm_mlp.hip", "lbm_surrogate.cpp", "lbm_persist_model.cpp"]
ARCH = "gfx950"


def build(verbose: bool = False, jobs: int = 8) -> str:
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    common = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-fopenmp",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(HERE, "..", "include")]
    objs, procs = [], []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        if not os.path.exists(src):
            continue
        obj = os.path.join(out_dir, s + ".o")
        cmd = common + (["-x", "hip"] if s.endswith(".hip") else []) + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), s))
        objs.append(obj)
        if len(procs) >= jobs:
            p, name = procs.pop(0)
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {name}")
    for p, name in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {name}")
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fopenmp", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
