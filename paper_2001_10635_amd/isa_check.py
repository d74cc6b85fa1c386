"""Build-time checks of the device assembly produced by build.py.

The kernels must never write through the scalar data cache: no scalar memory
stores, no scalar atomics, no write-back or discard of that cache.  This scans
the AMD assembly the compiler wrote for each source and fails the build if any
such instruction appears.  Host-side tooling only; nothing here runs on a GPU.
"""
import os

FORBIDDEN = ("s_store_", "s_atomic_", "s_dcache_wb", "s_dcache_discard", "s_buffer_store",
             "s_buffer_atomic", "s_scratch_store")


def check_device_asm(build_dir: str, src: str, arch: str) -> None:
    base = os.path.splitext(src)[0]
    path = os.path.join(build_dir, f"{base}-hip-amdgcn-amd-amdhsa-{arch}.s")
    if not os.path.exists(path):
        raise RuntimeError(f"device assembly {path} missing")
    with open(path) as f:
        bad = [ln for ln in f if any(t in ln for t in FORBIDDEN)]
    if bad:
        raise RuntimeError(f"{src}: scalar-cache write in device code:\n" + "".join(bad[:10]))
    # A kernel that reads the dispatch packet (the compiler asks for it when a
    # per-thread array with a lane-varying index is moved to LDS) makes every
    # wave read host memory at start-up; none of these kernels needs it.
    with open(path) as f:
        kern, uses = None, []
        for ln in f:
            t = ln.split()
            if len(t) >= 2 and t[0] == ".amdhsa_kernel":
                kern = t[1]
            elif len(t) >= 2 and t[0] == ".amdhsa_user_sgpr_dispatch_ptr" and t[1] == "1":
                uses.append(kern)
    if uses:
        raise RuntimeError(f"{src}: kernels reading the dispatch packet: " + ", ".join(uses[:5]))
