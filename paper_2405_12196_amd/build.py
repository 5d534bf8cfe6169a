"""Build the HIP library (gfx950) in-tree: paper_2405_12196_amd/libyastn.so.

Each translation unit is compiled to an object file in parallel (the kernel
instances of one arithmetic per unit), then linked into one shared library.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libyastn.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["device.hip", "host.cpp", "serve.cpp", "ops.hip", "svd.hip", "ctm.hip", "fermion.hip", "inst_f64.hip", "inst_f32d.hip", "inst_f32f.hip",
           "inst_bf16.hip", "inst_lds.hip", "inst_lds_norm.hip", "inst_ldsk.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Wall", "-Wno-unused-result",
    # packed FP32 VALU ops are disabled for every kernel of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _quiet(text):
    return "\n".join(l for l in text.splitlines()
                     if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)


def _compile(src):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r.returncode, _quiet(r.stdout + r.stderr), " ".join(cmd)


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = []
    for src, obj, rc, out, cmd in results:
        if verbose:
            print(cmd, flush=True)
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {src} ({rc}):\n{out}")
        if verbose and out.strip():
            print(out)
        objs.append(obj)
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + ["-o", LIB + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed ({r.returncode}):\n{_quiet(r.stdout + r.stderr)}")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
