"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer
and under ThreadSanitizer (CPU only): the host sources are rebuilt with the
sanitizer on their host pass only, linked with the built kernels' objects and a
driver that plans random batches of up to 250000 queries through
reach_plan_batch (several host threads for large plans).  The driver must
finish clean: no sanitizer report, every query scheduled once."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_10635_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2001_10635_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
KERNEL_OBJS = ["embed.o", "gb.o", "heat3d.o", "mc.o", "mc_noalloc.o", "batch.o"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-Wno-unused-value", "-Wno-unused-result"]


def build_driver(tmp, san):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    if not all(os.path.exists(os.path.join(BUILD, o)) for o in KERNEL_OBJS):
        pytest.skip("kernel objects not built (run __graft_entry__.build())")
    host = ["-Xarch_host", f"-fsanitize={san}", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in ("runtime.cpp", "server.cpp", "user.cpp",
                os.path.join(ROOT, "tests", "plan_sanitize_driver.cpp")):
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = os.path.join(tmp, os.path.basename(src) + ".o")
        subprocess.run([HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-x", "hip", *host,
                        "-c", path, "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    exe = os.path.join(tmp, "driver")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", f"-fsanitize={san}", *objs,
                    *[os.path.join(BUILD, o) for o in KERNEL_OBJS], "-o", exe,
                    "-lpthread", "-lhiprtc"], check=True, capture_output=True)
    return exe


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_planner_is_clean_under_sanitizers(tmp_path, san):
    exe = build_driver(str(tmp_path), san)
    env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "ALL OK" in r.stdout
    assert "Sanitizer" not in out and "runtime error" not in out, out[-3000:]
