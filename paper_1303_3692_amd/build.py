"""Compile libsamatch.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libsamatch.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = [
    "errors.cpp",
    "host_index.cpp",
    "dc3.cpp",
    "suffix_tree.cpp",
    "kernels.hip",
    "sa_construct.hip",
    "device.hip",
    "locate.hip",
    "tune.hip",
    "server.hip",
    "probe.hip",
]

ARCH = os.environ.get("SAMATCH_ARCH", "gfx950")
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}"]
# keep packed-fp32 instructions out of device code
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def build_id() -> str:
    """Hash of the sources of the tuned pipeline (kernels, batch enqueue,
    tuner): tuned launch settings are only reused for the same kernels."""
    import hashlib
    h = hashlib.sha256()
    for s in ["kernels.hip", "kernels.h", "radix_sort.h", "device.hip", "device_state.h", "tune.hip"]:
        h.update(open(os.path.join(CSRC, s), "rb").read())
    return h.hexdigest()[:12]


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [hipcc(), *COMMON, *DEVICE, *extra, "-c", path, "-o", obj]
    else:
        cmd = [hipcc(), *COMMON, *extra, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    """Compile every source and link libsamatch.so next to this file."""
    os.makedirs(BUILD, exist_ok=True)
    extra = list(extra or []) + [f'-DSAMATCH_BUILD_ID="{build_id()}"']
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT, file=sys.stderr)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
