"""Build the gfx950 shared library ``librbf_mi355x.so`` in-tree with hipcc.

Kernels whose results must be bit-identical to their mathematical definition
(node builder, neighbour search, weight solver) are compiled with
``-ffp-contract=off``; the sweep kernels may fuse multiply-adds.  Packed FP32
instructions are disabled for all device code.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librbf_mi355x.so")
BUILD_DIR = os.path.join(ROOT, "_build")
ARCH = os.environ.get("RBF_OFFLOAD_ARCH", "gfx950")

SOURCES = {
    "k_sweep.hip": [],
    "k_aux.hip": [],
    "k_sweep32.hip": [],
    "k_nodes.hip": ["-ffp-contract=off"],
    "k_knn.hip": ["-ffp-contract=off"],
    "k_weights.hip": ["-ffp-contract=off"],
    "k_weights_ns.hip": [],
    # null-space kernel sizes: row arrays indexed by fully unrolled loops
    "k_weights_ns_3d88.hip": ["-mllvm", "-pragma-unroll-threshold=2000000"],
    "k_weights_ns_3d64.hip": ["-mllvm", "-pragma-unroll-threshold=2000000"],
    "k_weights_ns_3d40.hip": ["-mllvm", "-pragma-unroll-threshold=2000000"],
    "k_weights_ns_2d.hip": ["-mllvm", "-pragma-unroll-threshold=2000000"],
    "k_transpose.hip": [],
    "rbf_api.cpp": [],
}

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result"]


def _compile(src, extra):
    obj = os.path.join(BUILD_DIR, src + ".o")
    lang = ["-x", "hip"]
    cmd = ["hipcc", *lang, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    return obj, out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        futs = [ex.submit(_compile, s, e) for s, e in SOURCES.items()]
        objs = []
        for f in futs:
            obj, out = f.result()
            if verbose and out.strip():
                print(out)
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
