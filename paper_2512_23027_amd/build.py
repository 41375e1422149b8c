"""Build the HIP/C++ library libsgw.so in-tree for gfx950 with hipcc."""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsgw.so")
SOURCES = ["setup.cpp", "coarse.cpp", "kernels.hip", "sgw.hip", "mlp.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def _jobs():
    """Parallel compiler processes: the CPU count, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n, int(os.environ.get("MAX_JOBS", "16"))))


def build(verbose=False):
    """Compile every source into libsgw.so (always rebuilds).  The generated
    SG-apply kernels (one translation unit per basis) compile in parallel
    with the hand-written sources."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    sys.path.insert(0, ROOT)
    from paper_2512_23027_amd import gen_k1
    gen_k1.generate()
    sources = SOURCES + gen_k1.sources()
    cmds, objs = [], []
    for src in sources:
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [hipcc] + [f for f in FLAGS if f != "-shared"] + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-pthread",
                   "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                   "-c", os.path.join(CSRC, src), "-o", obj]
        cmds.append(cmd)
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # longest first: the generated kernels of the largest bases
    order = sorted(range(len(cmds)), key=lambda i: -os.path.getsize(cmds[i][-3]))
    with ThreadPoolExecutor(_jobs()) as ex:
        for f in [ex.submit(run, cmds[i]) for i in order]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "-pthread", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
