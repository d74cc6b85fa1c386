"""Seeded synthetic workloads for interval reachability of the CTM and RD chains
and the 3-D heat grid.

This package only generates inputs (interval boxes, input intervals, query
streams).  It contains none of the method's arithmetic, so it feeds both the
FP64 oracle and the GPU library with bitwise-identical data.

The case studies follow the paper's sections on the n-link road traffic model
(cell transmission chain), on large sparse systems and on heat diffusion in a
cube; the paper publishes no
data sets for them, so every box here is synthetic, seeded, and regenerable
cell by cell (counter-based Philox4x64-10, see ``gen.c``).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libreach_workloads.so")
_lib = None

BASE_SEED = 20010635

# box recipes, same numbering as gen.c
CTM_RANDW, CTM_FIXEDW, SIN, HEAT_CORNER = 0, 1, 2, 3

# system kinds, same numbering as the C ABI
KIND_CTM, KIND_RD, KIND_LIN3, KIND_HEAT3D = 1, 2, 3, 4


def build(verbose: bool = False) -> str:
    """Compile gen.c into libreach_workloads.so (host code, OpenMP)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-std=c11", os.path.join(_HERE, "gen.c"), "-o", _SO + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    global _lib
    _lib = None
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.wl_philox4x64_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.wl_raw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                             ctypes.c_int64, ctypes.c_void_p]
        L.wl_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_void_p]
        L.wl_box.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                             ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                             ctypes.c_void_p, ctypes.c_void_p]
        L.wl_box.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().wl_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def raw(seed: int, stream: int, i0: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    if count:
        lib().wl_raw(seed, stream, i0, count, _p(out))
    return out


def uniform(seed: int, stream: int, i0: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    if count:
        lib().wl_uniform(seed, stream, i0, count, _p(out))
    return out


def box(recipe: int, prm, seed: int, n: int, i0: int = 0, count: int | None = None,
        dtype=np.float64, out=None):
    """Cells [i0, i0+count) of the seeded box; returns (lo, hi) numpy arrays."""
    if count is None:
        count = n - i0
    dtype = np.dtype(dtype)
    prm_a = np.zeros(8, dtype=np.float64)
    prm_a[: len(prm)] = prm
    if out is None:
        lo = np.empty(count, dtype=dtype)
        hi = np.empty(count, dtype=dtype)
    else:
        lo, hi = out
        assert lo.dtype == dtype and hi.dtype == dtype and lo.size >= count and hi.size >= count
    rc = lib().wl_box(recipe, _p(prm_a), seed, n, i0, count, 1 if dtype == np.float32 else 0,
                      _p(lo), _p(hi))
    if rc != 0:
        raise ValueError("wl_box: bad recipe or range")
    return lo, hi


# ---------------------------------------------------------------- systems

CTM_PRM = (0.5, 1.0 / 6.0, 40.0, 20.0)  # v, w, c, q
RD_PRM = (1.0,)                          # h
CTM_BOX_A, CTM_BOX_D = 12.0, 2.0         # 0.3*c and 0.05*c for c = 40
RD_BOX_W = 0.02
RD_U = (-0.1, 0.1)


@dataclass
class Problem:
    """One reachability problem: a system, its box, inputs and horizon."""
    name: str
    kind: int
    n: int
    prm: tuple
    dtype: type
    recipe: int
    box_prm: tuple
    seed: int
    dt: float
    nsteps: int
    t0: float = 0.0
    n_in: int = 0
    p_lo: tuple = ()
    p_hi: tuple = ()
    m: int = 0                     # Monte Carlo samples (0: embedding only)
    extra: dict = field(default_factory=dict)

    def box(self, i0: int = 0, count: int | None = None, out=None):
        return box(self.recipe, self.box_prm, self.seed, self.n, i0, count, self.dtype, out)

    def inputs(self):
        """(p_lo, p_hi) arrays of length n_in (None when n_in = 0)."""
        if self.n_in == 0:
            return None, None
        return (np.array(self.p_lo, dtype=self.dtype), np.array(self.p_hi, dtype=self.dtype))


def ctm64_f64() -> Problem:
    """Cell-transmission chain, n = 64, FP64, dt = 0.01, 100 RK4 steps, with a
    1000-sample Monte Carlo check."""
    return Problem("ctm64_f64", KIND_CTM, 64, CTM_PRM, np.float64, CTM_RANDW,
                   (CTM_BOX_A, CTM_BOX_D), BASE_SEED + 0, 0.01, 100, m=1000)


def rd_2p26_f64() -> Problem:
    """Reaction-diffusion chain, n = 2^26, FP64, input u in [-0.1, 0.1],
    dt = 0.1, 1000 RK4 steps."""
    return Problem("rd_2^26_f64", KIND_RD, 1 << 26, RD_PRM, np.float64, SIN, (RD_BOX_W,),
                   BASE_SEED + 1, 0.1, 1000, n_in=1, p_lo=(RD_U[0],), p_hi=(RD_U[1],))


def ctm_2p31_f32() -> Problem:
    """Cell-transmission chain, n = 2^31, FP32, dt = 0.01, 200 RK4 steps."""
    return Problem("ctm_2^31_f32", KIND_CTM, 1 << 31, CTM_PRM, np.float32, CTM_RANDW,
                   (CTM_BOX_A, CTM_BOX_D), BASE_SEED + 2, 0.01, 200)


def mc_ctm4096_f32() -> Problem:
    """Monte Carlo on the cell-transmission chain, n = 4096, box width 0.05c,
    2^20 samples, FP32, dt = 0.01, 500 RK4 steps."""
    return Problem("mc_ctm4096_f32", KIND_CTM, 4096, CTM_PRM, np.float32, CTM_FIXEDW,
                   (CTM_BOX_A, CTM_BOX_D), BASE_SEED + 3, 0.01, 500, m=1 << 20)


def serve_mix_f64() -> Problem:
    """Parameters of the served query mix: 10^5 queries at 5e4/s (see
    query_stream for the draws)."""
    return Problem("serve_mix_f64", KIND_CTM, 512, CTM_PRM, np.float64, CTM_RANDW,
                   (CTM_BOX_A, CTM_BOX_D), BASE_SEED + 4, 0.01, 1000,
                   extra=dict(nq=100000, rate=5.0e4))


# 3-D heat grid (heat diffusion case study): unit cube, l cells per edge,
# spacing 1/l.  The paper prints no diffusivity; HEAT_ALPHA keeps classical
# RK4 at dt = 0.02 stable on the 1000^3 grid (spectral radius of the grid
# operator times dt = 12 alpha l^2 dt = 2.4 < 2.78, RK4's real-axis limit).
HEAT_ALPHA = 1.0e-5
HEAT_BOX = (0.5, 1.0, 0.1, 0.01)     # heated corner fraction, T, half-width, cold width


def heat3d_problem(nx: int, ny: int, nz: int, seed: int, nsteps: int, dtype=np.float64,
                   dt: float = 0.02, alpha: float = HEAT_ALPHA, dx: float | None = None) -> Problem:
    """A 3-D heat grid with the heated-corner box recipe."""
    dx = 1.0 / max(nx, ny, nz) if dx is None else dx
    return Problem(f"heat3d_{nx}x{ny}x{nz}", KIND_HEAT3D, nx * ny * nz,
                   (float(nx), float(ny), float(nz), alpha, dx), dtype, HEAT_CORNER,
                   (float(nx), float(ny), float(nz)) + HEAT_BOX, seed, dt, nsteps)


def heat3d_1000_f64() -> Problem:
    """The heat diffusion case study at its stated size: l = 1000 (n = 10^9),
    FP64, [t0, t1] = [0, 20] with dt = 0.02 (1000 RK4 steps)."""
    p = heat3d_problem(1000, 1000, 1000, BASE_SEED + 5, 1000)
    p.name = "heat3d_1000^3_f64"
    return p


def small_problem(kind: int, n: int, seed: int, nsteps: int, dtype=np.float64,
                  dt: float | None = None) -> Problem:
    """A CTM or RD chain of any size with the benchmark's box recipe."""
    if kind == KIND_CTM:
        return Problem(f"ctm{n}", KIND_CTM, n, CTM_PRM, dtype, CTM_RANDW,
                       (CTM_BOX_A, CTM_BOX_D), seed, 0.01 if dt is None else dt, nsteps)
    if kind == KIND_RD:
        return Problem(f"rd{n}", KIND_RD, n, RD_PRM, dtype, SIN, (RD_BOX_W,), seed,
                       0.1 if dt is None else dt, nsteps, n_in=1,
                       p_lo=(RD_U[0],), p_hi=(RD_U[1],))
    raise KeyError(kind)


# ---------------------------------------------------------------- query stream

@dataclass
class Query:
    idx: int
    arrival: float      # seconds since the stream start
    problem: Problem


def query_stream(nq: int, rate: float, seed: int = BASE_SEED + 4,
                 n_range=(4, 512), steps_range=(10, 1000)) -> list[Query]:
    """Poisson arrivals of CTM / RD queries with log-uniform size and horizon.

    Draw q uses stream 3 at indices 5q .. 5q+3: inter-arrival gap (exponential
    with the given rate), kind (CTM or RD with probability 1/2 each), n and the
    number of RK4 steps (log-uniform on the given ranges).  Query q's box is
    generated with seed + 1 + q, so each query is reproducible on its own.
    """
    u = uniform(seed, 3, 0, 5 * nq).reshape(nq, 5)
    t = 0.0
    out = []
    lo_n, hi_n = n_range
    lo_s, hi_s = steps_range
    for q in range(nq):
        t += -math.log1p(-u[q, 0]) / rate
        kind = KIND_CTM if u[q, 1] < 0.5 else KIND_RD
        n = min(hi_n, int(math.floor(math.exp(u[q, 2] * math.log((hi_n + 1) / lo_n)) * lo_n)))
        ns = min(hi_s, int(math.floor(math.exp(u[q, 3] * math.log((hi_s + 1) / lo_s)) * lo_s)))
        out.append(Query(q, t, small_problem(kind, n, seed + 1 + q, ns)))
    return out
