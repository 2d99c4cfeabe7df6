"""Build libvi.so (HIP, gfx950) in-tree with hipcc, and the benchmark's L2
probe libvi_probe.so beside it.

    python -m paper_2008_06134_amd.build

Every HIP source is compiled with packed-FP32 instruction selection turned
off (``-Xclang -target-feature -Xclang -packed-fp32-ops``); the host pass
warns that it does not know that feature, which is harmless.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libvi.so")
# the benchmark's probes (L2 reads, the build's store pattern), a library of its own that only bench.py loads
PROBE_SRC, PROBE_OUT = "vi_probe.hip", os.path.join(HERE, "libvi_probe.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["vi_api.hip", "vi_build.hip", "vi_render.hip", "vi_layout.hip", "vi_sched.cpp", "vi_server.hip"]
ARCH = os.environ.get("VI_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: libvi needs the ROCm toolchain")


def flags() -> list:
    # VI_BUILD_DEFINES: extra -D options for experiments with the kernels'
    # compile-time switches (e.g. "-DVI_RENDER_COMPACT=1"); empty by default
    extra = os.environ.get("VI_BUILD_DEFINES", "").split()
    if any(not e.startswith("-D") for e in extra):
        raise RuntimeError("VI_BUILD_DEFINES takes -D options only")
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), *extra]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()

    def compile_one(src):
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [cc, *flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    build_probe(cc)
    return OUT


def build_probe(cc: str) -> str:
    tmp = PROBE_OUT + ".tmp"
    cmd = [cc, *flags(), "-shared", "-o", tmp, os.path.join(CSRC, PROBE_SRC)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {PROBE_SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PROBE_OUT)
    return PROBE_OUT


if __name__ == "__main__":
    print(build(verbose=True))
