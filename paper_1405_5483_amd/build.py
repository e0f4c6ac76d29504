"""Builds ``libmag.so`` (HIP kernels + C ABI) for gfx950 with hipcc.

Usage: ``python -m paper_1405_5483_amd.build`` (always recompiles).
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmag.so")
BUILD_DIR = os.path.join(ROOT, "_build")
ARCH = os.environ.get("MAG_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    cand = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cand):
        raise RuntimeError("hipcc not found; ROCm is required to build the MAG library")
    return cand


def common_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # packed fp32 instructions are kept out of every build
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-Wall", "-Wno-unused-function",
    ]


def _compile(job) -> str:
    src, defines = job
    tag = "".join(f".{d.replace('=', '')}" for d in defines)
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + tag + ".o")
    cmd = [hipcc(), "-x", "hip", "-c", src, "-o", obj] + common_flags() + [f"-D{d}" for d in defines]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = []
    for src in sources:
        if os.path.basename(src) == "scan.hip":       # one object per q-gram length
            jobs += [(src, [f"MAG_SCAN_Q={q}"]) for q in range(1, 9)]
        else:
            jobs.append((src, []))
    workers = max(1, min(16, os.cpu_count() or 1, len(jobs)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, jobs))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
