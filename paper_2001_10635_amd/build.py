"""Build libreach.so (HIP kernels + C-ABI runtime) for gfx950 with hipcc.

Each source compiles to its own object in parallel; the shared library links
them.  The device assembly of each object is kept and checked by isa_check.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
SO = os.path.join(HERE, "libreach.so")
# the HBM ceiling probe of the benchmark, a library of its own
PROBE_SRC = "hbm_probe.hip"
PROBE_SO = os.path.join(HERE, "libreach_probe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["embed.hip", "gb.hip", "heat3d.hip", "mc.hip", "mc_noalloc.hip", "batch.hip",
           "runtime.cpp", "server.cpp", "user.cpp"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-Wno-unused-value", "-Wno-unused-result"]


def _obj(src: str) -> str:
    return os.path.join(BUILD, os.path.splitext(src)[0] + ".o")


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC, *COMMON, *lang, "-save-temps=obj", "-c", path, "-o", _obj(src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return _obj(src)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES + [PROBE_SRC]))
    probe_obj = objs.pop()
    from .isa_check import check_device_asm
    for src in SOURCES + [PROBE_SRC]:
        check_device_asm(BUILD, src, ARCH)
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", SO + ".tmp",
           "-lpthread", "-lhiprtc"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(SO + ".tmp", SO)
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", probe_obj, "-o", PROBE_SO + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(PROBE_SO + ".tmp", PROBE_SO)
    if verbose:
        print("built", SO, "and", PROBE_SO)
    return SO


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2001_10635_amd.build import build as _b
    _b(verbose=True)
    sys.exit(0)
