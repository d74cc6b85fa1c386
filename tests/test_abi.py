"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/reach.h declares, and its host-only logic holds."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "reach.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(reach_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def R():
    import paper_2001_10635_amd as R
    if not os.path.exists(R.LIB_PATH):
        pytest.fail("libreach.so is not built (run __graft_entry__.build())")
    return R


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ["reach_embed_rk4", "reach_montecarlo", "reach_submit", "reach_poll",
                 "reach_ctx_create", "reach_sync", "reach_mc_samples", "reach_embed_rk4_batch"]:
        assert name in fns


def test_library_exports_every_declared_symbol(R):
    L = R.lib()
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing


def test_struct_layouts_match_header(R):
    assert ctypes.sizeof(R.reach_system) == 4 + 4 + 8 + 8 + 64
    assert ctypes.sizeof(R.reach_query) == ctypes.sizeof(R.reach_system) + 8 + 6 * 8 + 3 * 8


def test_mc_sample_count_host_function(R):
    """reach_mc_samples is the least m with 2n exp(-eps m / (2n)) <= delta."""
    for n, eps, delta in [(1, 0.1, 0.05), (64, 0.01, 0.01), (4096, 0.05, 1e-3)]:
        m = R.reach_mc_samples(n, eps, delta)
        assert 2 * n * math.exp(-eps * m / (2 * n)) <= delta * (1 + 1e-12)
        assert 2 * n * math.exp(-eps * (m - 1) / (2 * n)) > delta * (1 - 1e-9)
    assert R.reach_mc_samples(0, 0.1, 0.1) == -1
    assert R.reach_mc_samples(5, 1.0, 0.1) == -1
    assert R.reach_mc_samples(5, 0.1, 0.0) == -1


def test_batch_workspace_size_is_monotone(R):
    a, b = R.reach_batch_workspace_bytes(10), R.reach_batch_workspace_bytes(1000)
    assert 0 < a < b
    assert R.reach_batch_workspace_bytes(-1) == ctypes.c_size_t(-1).value


def test_context_needs_a_device(R):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(R.ReachError) as e:
        R.reach_ctx_create(0)
    assert e.value.status == R.REACH_E_DEVICE


def test_null_context_is_rejected(R):
    L = R.lib()
    assert L.reach_sync(None, None) == R.REACH_E_INVAL
    assert L.reach_set_option(None, b"embed.K", 1) == R.REACH_E_INVAL
    assert L.reach_embed_rk4_batch(None, None, 0, None, 0, None) == R.REACH_E_INVAL
    assert L.reach_submit(None, None, None) == R.REACH_E_BUSY


def test_noalloc_scratch_size_and_null_context(R):
    """The no-allocation Monte Carlo's fixed scratch array is 64 MiB; a NULL
    context is rejected before anything touches a device."""
    L = R.lib()
    assert R.reach_noalloc_scratch_bytes() == 64 << 20
    assert L.reach_montecarlo_noalloc(None, None, 0, None, None, None, None, 0.0, 0.1, 1, 0, 1,
                                      0, None, None, None) == R.REACH_E_INVAL


def test_step_count_from_horizon(R):
    """nsteps = round((t1 - t0) / dt); a horizon that is not a whole number of
    steps (beyond 1e-9 relative) is rejected."""
    assert R.steps_between(0.0, 1.0, 0.01) == 100
    assert R.steps_between(0.0, 20.0, 0.02) == 1000
    assert R.steps_between(2.5, 2.5, 0.1) == 0
    with pytest.raises(ValueError):
        R.steps_between(0.0, 1.0, 0.3)
    with pytest.raises(ValueError):
        R.steps_between(1.0, 0.0, 0.1)
    assert R._nsteps(None, 0.0, 1.0, 0.1) == 10
    with pytest.raises(ValueError):
        R._nsteps(9, 0.0, 1.0, 0.1)


def test_build_rejects_kernels_reading_the_dispatch_packet(tmp_path):
    """The build's assembly check fails a source whose kernel asks for the
    dispatch packet (every wave would read host memory at start-up) and passes
    one that does not; the library's own assembly passes it."""
    from paper_2001_10635_amd.isa_check import check_device_asm
    arch = "gfx950"

    def write(name, flag):
        (tmp_path / f"{name}-hip-amdgcn-amd-amdhsa-{arch}.s").write_text(
            f"\t.amdhsa_kernel k_{name}\n\t\t.amdhsa_user_sgpr_dispatch_ptr {flag}\n"
            "\t.end_amdhsa_kernel\n")

    write("good", 0)
    write("bad", 1)
    check_device_asm(str(tmp_path), "good.hip", arch)
    with pytest.raises(RuntimeError, match="dispatch packet"):
        check_device_asm(str(tmp_path), "bad.hip", arch)
    build = os.path.join(ROOT, "paper_2001_10635_amd", "_build")
    if os.path.exists(os.path.join(build, f"mc-hip-amdgcn-amd-amdhsa-{arch}.s")):
        check_device_asm(build, "mc.hip", arch)
