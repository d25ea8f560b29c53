"""Build libbvs.so (gfx950) from the sources in this folder.

Every source is compiled by hipcc for gfx950 only and linked into
paper_2412_03301_amd/libbvs.so.  Packed FP32 instructions are disabled
(`-packed-fp32-ops`), as required for every HIP translation unit here.
Usage: python -m paper_2412_03301_amd.csrc.build [-j N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_obj")
OUT = os.path.join(PKG, "libbvs.so")

SOURCES = ["capi.cpp", "k_encode.hip", "k_filter.hip", "k_sliced.hip", "k_haus.hip", "k_batch.hip", "k_lowp.hip", "k_learn.hip",
           "k_full.hip", "k_lists.hip"]
HEADERS = ["device.h", "launch.h", "haus_core.h", "wta.h", os.path.join(INCLUDE, "bvs.h")]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-mcode-object-version=5",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            f"-I{INCLUDE}", f"-I{HERE}", "-Wno-unused-result"]


def compile_one(src: str) -> str:
    os.makedirs(OBJ, exist_ok=True)
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *common_flags(), "-c", os.path.join(HERE, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-xhip")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def _fresh(src: str) -> bool:
    """The object of src is newer than src and every header."""
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    if not os.path.exists(obj):
        return False
    deps = [os.path.join(HERE, src)] + [h if os.path.isabs(h) else os.path.join(HERE, h) for h in HEADERS]
    return all(os.path.getmtime(obj) > os.path.getmtime(d) for d in deps)


def build(jobs: int = 4, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental: only those whose object is stale)
    and link libbvs.so."""
    def one(src):
        if incremental and _fresh(src):
            return os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        return compile_one(src)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-L/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=min(8, os.cpu_count() or 4))
    ap.add_argument("--incremental", action="store_true", help="recompile only sources with stale objects")
    a = ap.parse_args()
    try:
        build(a.j, verbose=True, incremental=a.incremental)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
