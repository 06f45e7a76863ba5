"""Build the gfx950 HIP library libeph.so in-tree (hipcc, no JIT).

Each source is compiled to an object of its own, in parallel, then the
objects are linked into one shared library.  Every call recompiles every
source.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libeph.so")
OBJ_DIR = os.path.join(ROOT, "_build", "obj")

HIPCC = "/opt/rocm/bin/hipcc"
# packed FP32 instructions stay off: the feature flag keeps hipcc -O3 from
# forming them out of ordinary float code
COMMON = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def compile_command(src, obj, debug=False, defines=()):
    cmd = [HIPCC, "-c"] + COMMON + ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
                                     "-o", obj, src]
    if debug:
        cmd.insert(1, "-g")
    for d in defines:
        cmd.insert(1, "-D" + d)
    return cmd


def hipcc_command(out=LIB, debug=False, defines=()):
    """One-line equivalent of the build (all sources in one hipcc call)."""
    cmd = [HIPCC, "-shared"] + COMMON + ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
                                         "-o", out] + sources()
    for d in defines:
        cmd.insert(1, "-D" + d)
    return cmd


def build(verbose=False, out=LIB, defines=(), jobs=None):
    srcs = sources()
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(os.path.basename(s))[0] + ".o") for s in srcs]
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))

    def one(pair):
        src, obj = pair
        cmd = compile_command(src, obj, defines=defines)
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return src, r.returncode, r.stdout

    failed = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, rc, log in ex.map(one, zip(srcs, objs)):
            noise = [l for l in log.splitlines() if "packed-fp32-ops" not in l]
            if noise and (verbose or rc):
                print("\n".join(noise), flush=True)
            if rc:
                failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed on: " + ", ".join(os.path.basename(f) for f in failed))
    tmp = out + ".tmp"
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, out)
    return out


def clean():
    shutil.rmtree(OBJ_DIR, ignore_errors=True)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
