"""Build librdcnn.so (the HIP kernels and the C ABI) in-tree for gfx950.

Run ``python -m paper_2102_10340_amd.build`` (``--changed``: recompile only
sources older than their inputs).  Every source is compiled with:
  -ffp-contract=off                    no fusion beyond the explicit fmaf calls,
                                       so the float32 rounding order is fixed
  -fno-gpu-flush-denormals-to-zero     IEEE denormals, as on the host
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                       no packed FP32 instructions
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librdcnn.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["rd_api.hip", "rd_forward.hip", "rd_adjoint.hip", "rd_batch.hip", "rd_stats.hip",
           "rd_models.hip", "rd_fwd_r0c1.hip", "rd_fwd_r0c2.hip", "rd_fwd_r0c4.hip",
           "rd_fwd_r1c1.hip", "rd_fwd_r1c2.hip", "rd_fwd_r1c4.hip", "rd_fwd_r23.hip",
           "rd_adj_plain.hip", "rd_adj_pair.hip", "rd_adj_batch.hip", "rd_batch_r0.hip",
           "rd_batch_rec.hip"]
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _deps(path: str, seen=None) -> set:
    """The file and every header of csrc/ or include/ it includes, transitively."""
    import re
    seen = set() if seen is None else seen
    if path in seen:
        return seen
    seen.add(path)
    with open(path) as f:
        for name in re.findall(r'^\s*#\s*include\s+"([^"]+)"', f.read(), flags=re.M):
            for d in (CSRC, INCLUDE):
                q = os.path.join(d, name)
                if os.path.exists(q):
                    _deps(q, seen)
                    break
    return seen


def _stale(obj: str, src: str) -> bool:
    """An object is stale if it is missing or older than its source or a
    header the source includes."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in _deps(src))


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force=False: only those older than their inputs)
    and link librdcnn.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    hipcc = _hipcc()

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        if not force and not _stale(obj, os.path.join(CSRC, src)):
            return obj
        cmd = [hipcc, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    # the largest sources first, so they do not start last
    order = sorted(SOURCES, key=lambda f: -os.path.getsize(os.path.join(CSRC, f)))
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        done = dict(zip(order, ex.map(compile_one, order)))
    objs = [done[f] for f in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--changed" not in sys.argv))
