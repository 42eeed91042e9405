"""Builds libsoprop.so (the HIP kernels + C ABI) in-tree for gfx950.

    python -m paper_1903_04946_amd.build            # incremental
    python -m paper_1903_04946_amd.build --force    # rebuild everything

Each translation unit is compiled with hipcc to an object under _build/ and
the objects are linked into paper_1903_04946_amd/libsoprop.so.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsoprop.so")
SOURCES = ["kernels_3d.hip", "kernels_batch3d.hip", "kernels_batch1d.hip", "kernels_1d.hip",
           "kernels_aux.hip", "kernels_interp.hip", "kernels_trap.hip", "kernels_trap3d.hip",
           "plan.cpp", "batch.cpp"]
HEADERS = ["fft_core.hpp", "internal.hpp", "body_1d.hpp", "body_1d_w4.hpp", "passes_3d.hpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-std=c++20", "-O3", "--offload-arch=gfx950", "-fPIC",
         # never emit packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _deps_mtime() -> float:
    paths = [os.path.join(CSRC, h) for h in HEADERS]
    paths.append(os.path.join(ROOT, "include", "soprop.h"))
    return max(os.path.getmtime(p) for p in paths)


def _compile(src: str, force: bool) -> str:
    obj = os.path.join(BUILD, src + ".o")
    srcp = os.path.join(CSRC, src)
    if (not force and os.path.exists(obj)
            and os.path.getmtime(obj) >= max(os.path.getmtime(srcp), _deps_mtime())):
        return obj
    cmd = [HIPCC, *FLAGS, "-c", srcp, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(force: bool = False, jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), SOURCES))
    if (force or not os.path.exists(LIB)
            or os.path.getmtime(LIB) < max(os.path.getmtime(o) for o in objs)):
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(LIB + ".tmp", LIB)
    return LIB


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", "--jobs", type=int, default=6)
    a = ap.parse_args(argv)
    print(build(a.force, a.jobs))
    return 0


if __name__ == "__main__":
    sys.exit(main())
