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
    "noalloc.hip",
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


# Sanitizer builds of the host code, for the CPU tests: every source
# compiled for the host only (no device code, so no kernel can launch), each
# -fsanitize= applying to the host pass only.  The sanitizer's runtime is not
# linked in: the process that loads the library preloads it (runtime_path).
SANITIZERS = {
    "address": ["-fsanitize=address", "-fsanitize=undefined"],
    "thread": ["-fsanitize=thread"],
}


def runtime_path(kind: str) -> str:
    """The clang sanitizer runtime to preload for a build of `kind`
    (the address runtime carries the undefined-behaviour handlers too)."""
    r = subprocess.run([hipcc(), "--print-resource-dir"], capture_output=True, text=True)
    res = r.stdout.strip() if r.returncode == 0 else ""
    name = {"address": "libclang_rt.asan-x86_64.so", "thread": "libclang_rt.tsan-x86_64.so"}[kind]
    path = os.path.join(res, "lib", "linux", name)
    if not os.path.exists(path):
        raise RuntimeError(f"sanitizer runtime {name} not found under {res}")
    return path


def build_sanitized(kind: str) -> str:
    """Host-only library instrumented with the `kind` sanitizer(s); returns
    its path (under _build/, never next to the product library)."""
    out_dir = os.path.join(BUILD, f"san_{kind}")
    os.makedirs(out_dir, exist_ok=True)
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "--cuda-host-only"]
    for f in SANITIZERS[kind]:
        flags += ["-Xarch_host", f]
    base = [f for f in COMMON if f != "-O3"]

    def one(src: str) -> str:
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc(), *base, *flags, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(one, SOURCES))
    # A host-only object still names the device image its source would
    # embed (__hip_fatbin_<id>).  This build has none: each is defined as an
    # empty image, so the library loads on a machine without a GPU, and no
    # kernel exists to launch.
    names = set()
    for o in objs:
        r = subprocess.run(["nm", "-u", o], capture_output=True, text=True, check=True)
        names.update(w for line in r.stdout.splitlines() for w in line.split() if w.startswith("__hip_fatbin_"))
    stub = os.path.join(out_dir, "no_device_images.c")
    with open(stub, "w") as f:
        for nm in sorted(names):
            f.write(f"const unsigned char {nm}[64] = {{0}};\n")
    stub_obj = stub + ".o"
    subprocess.run(["gcc", "-fPIC", "-c", stub, "-o", stub_obj], check=True)
    objs.append(stub_obj)
    out = os.path.join(out_dir, "libsamatch.so")
    cmd = [hipcc(), "-shared", "-fPIC", "-o", out, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


if __name__ == "__main__":
    build(verbose=True)
