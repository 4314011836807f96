"""Build libmirt.so (the C-ABI ray tracing library) for gfx950 with hipcc.

Usage: python -m paper_1504_03151_amd.csrc.build [--jobs N] [--verbose]
Writes paper_1504_03151_amd/libmirt.so (in-tree, so it travels with the repo).
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
OUT = os.path.join(PKG, "libmirt.so")
OBJDIR = os.path.join(ROOT, "_build", "mirt")

SOURCES = ["scene.cpp", "render.cpp", "mlp.cpp", "refit.cpp"]
HEADERS = ["rt_common.h", "mirt_internal.h", "bvh_quant.h", os.path.join("..", "..", "include", "mirt.h")]

ARCH = os.environ.get("MIRT_ARCH", "gfx950")
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-x", "hip",
    "-munsafe-fp-atomics",                 # hardware float atomics on device memory
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc", "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libmirt.so)")


def _stale(obj: str, src: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(HERE, h) for h in HEADERS]
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def build(jobs: int = 0, verbose: bool = False, force: bool = True, out: str = OUT, objdir: str = OBJDIR) -> str:
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    objs, cmds = [], []
    for s in SOURCES:
        src = os.path.join(HERE, s)
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        objs.append(obj)
        if force or _stale(obj, src):
            cmds.append([cc] + COMMON + ["-c", src, "-o", obj])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)

    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(run, cmds))
    tmp = out + ".tmp"
    link = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lamdhip64"]
    run(link)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=0)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("--out", default=OUT, help="library path (default: in-tree libmirt.so)")
    ap.add_argument("--objdir", default=OBJDIR)
    a = ap.parse_args()
    print(build(a.jobs, a.verbose, force=not a.incremental, out=os.path.abspath(a.out), objdir=a.objdir))
