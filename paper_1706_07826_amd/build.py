"""Build libspvar.so (HIP for gfx950) in-tree with hipcc, and its race-detection
variant libspvar_shadow.so (SPV_LDS_SHADOW=1).  Each source is compiled on its own
(in parallel, objects under _build/), then linked."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libspvar.so")
SHADOW_LIB = os.path.join(HERE, "libspvar_shadow.so")
OBJ_DIR = os.path.join(ROOT, "_build")
ARCH = os.environ.get("SPVAR_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unknown-warning-option",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]
VARIANTS = {"default": (LIB, []), "shadow": (SHADOW_LIB, ["-DSPV_LDS_SHADOW=1"])}


def sources():
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    srcs += sorted(glob.glob(os.path.join(HERE, "csrc", "*.cpp")))
    return srcs


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise subprocess.CalledProcessError(p.returncode, cmd, p.stdout, p.stderr)
    if verbose and p.stderr.strip():
        print(p.stderr, end="", flush=True)


def build(verbose=False, variants=("default", "shadow"), jobs=None):
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    plan = []
    for v in variants:
        out_dir = os.path.join(OBJ_DIR, v)
        os.makedirs(out_dir, exist_ok=True)
        for src in sources():
            obj = os.path.join(out_dir, os.path.basename(src) + ".o")
            plan.append((v, obj, ["hipcc", *FLAGS, *VARIANTS[v][1], "-c", "-o", obj, src]))
    # the longest sources first, so the pool ends together
    plan.sort(key=lambda t: -os.path.getsize(t[2][-1]))
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda t: _run(t[2], verbose), plan))
    built = []
    for v in variants:
        lib = VARIANTS[v][0]
        objs = [o for (w, o, _) in plan if w == v]
        tmp = lib + ".tmp"
        _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *sorted(objs)], verbose)
        os.replace(tmp, lib)
        built.append(lib)
    return built


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
