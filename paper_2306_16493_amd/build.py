"""Build the gfx950 HIP library libeph.so in-tree (hipcc, no JIT)."""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libeph.so")


def hipcc_command(out=LIB, arch="gfx950", debug=False, defines=()):
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    cmd = ["/opt/rocm/bin/hipcc", "-shared", "-fPIC", "-std=c++17", "-O3",
           "--offload-arch=" + arch,
           # packed FP32 instructions stay off (see the design notes)
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", out] + srcs
    if debug:
        cmd.insert(1, "-g")
    for d in defines:
        cmd.insert(1, "-D" + d)
    return cmd


def build(verbose=False, out=LIB, defines=()):
    cmd = hipcc_command(out=out, defines=defines)
    if verbose:
        print(" ".join(cmd), flush=True)
    tmp = out + ".tmp"
    cmd[cmd.index("-o") + 1] = tmp
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
