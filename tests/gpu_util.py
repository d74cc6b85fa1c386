"""Shared helpers of the GPU tests: tolerance check, tensors from workloads."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

RTOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5}

gpu = pytest.mark.gpu


def have_gpu() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def say(msg: str) -> None:
    """Name the case before a GPU step, so a fault report says which one."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def assert_rel(got, ref, rtol, what=""):
    """|got - ref| <= rtol * max(|ref|, 1) elementwise (states cross 0)."""
    g = np.asarray(got, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    assert g.shape == r.shape, f"{what}: shape {g.shape} vs {r.shape}"
    assert np.all(np.isfinite(g)), f"{what}: non-finite GPU values"
    err = (np.abs(g - r) / np.maximum(np.abs(r), 1.0)).ravel()
    i = int(np.argmax(err)) if err.size else 0
    assert err.size == 0 or err[i] <= rtol, \
        f"{what}: rel err {err[i]:.3e} > {rtol:.0e} at {i} (gpu {g.flat[i]!r}, oracle {r.flat[i]!r})"
    return float(err.max()) if err.size else 0.0


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()
