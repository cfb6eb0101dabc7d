"""Build the gfx950 library libjjacobi.so in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libjjacobi.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("jj_kernels.hip", "jj_pivot.hip", "jj_batched.hip", "jj_frontend.hip",
                                                                   "jj_three.hip", "jj_solver.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (they are never written by hand either)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build(out=SO, verbose=False):
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out_lines = [l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l and "warnings generated" not in l]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(out_lines))
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
