"""FP64 CPU oracle (test infrastructure only).

A plain, slow, obviously correct implementation of what the GPU library
computes, written from the PIRK paper (arXiv 2001.10635): the mixed-monotone
embedding system integrated by classical RK4 (Sec. 2.1, Algorithms 1 and 3)
and the Monte Carlo batch of sampled RK4 trajectories with its per-dimension
min / max (Sec. 2.1, Algorithm 4), the growth-bound method (Algorithm 2), on
the chain systems and the 3-D heat diffusion case study (Sec. 5).  See ``oracle.c`` for the equations.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the GPU library and does not import it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

CTM, RD, LIN3, HEAT3D, USER = 1, 2, 3, 4, 5


def build(verbose: bool = False) -> str:
    """Compile oracle.c (C99, OpenMP, FP64, no FP contraction)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-std=gnu99", os.path.join(_HERE, "oracle.c"),
           "-o", _SO + ".tmp", "-lm"]
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
        vp, i64, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.or_philox4x64_10.argtypes = [vp, vp, vp]
        L.or_uniform.argtypes = [ctypes.c_uint64, i64, i64, ctypes.c_int]
        L.or_uniform.restype = d
        L.or_rhs.argtypes = [ctypes.c_int, vp, i64, i64, i64, i64, vp, vp, vp, vp,
                             ctypes.c_int, vp]
        L.or_embed_rk4.argtypes = [ctypes.c_int, vp, i64, i64, i64, i64, vp, vp, vp, vp,
                                   d, d, i64, vp, vp]
        L.or_embed_rk4.restype = ctypes.c_int
        L.or_embed_rk4_grid.argtypes = [vp, vp, vp, vp, vp, d, i64, vp, vp]
        L.or_embed_rk4_grid.restype = ctypes.c_int
        L.or_embed_rk4_user.argtypes = [vp, vp, i64, i64, i64, i64, vp, vp, vp, vp, d, i64,
                                        vp, vp]
        L.or_embed_rk4_user.restype = ctypes.c_int
        L.or_f_rk4_user.argtypes = [vp, vp, i64, i64, vp, vp, d, i64, vp]
        L.or_montecarlo_user.argtypes = [vp, vp, i64, i64, vp, vp, vp, vp, d, i64, i64, i64,
                                         ctypes.c_uint64, ctypes.c_int, vp, vp, vp]
        L.or_montecarlo_user.restype = ctypes.c_int
        L.or_f_rk4_user.restype = ctypes.c_int
        L.or_f_rk4.argtypes = [ctypes.c_int, vp, i64, i64, vp, vp, d, d, i64, vp]
        L.or_f_rk4.restype = ctypes.c_int
        L.or_montecarlo.argtypes = [ctypes.c_int, vp, i64, i64, vp, vp, vp, vp, d, d, i64,
                                    i64, i64, ctypes.c_uint64, ctypes.c_int, vp, vp, vp]
        L.or_montecarlo.restype = ctypes.c_int
        L.or_growth_bound.argtypes = [ctypes.c_int, vp, i64, i64, i64, i64, vp, vp, vp, vp,
                                      d, d, i64, vp, vp]
        L.or_growth_bound.restype = ctypes.c_int
        L.or_contraction_matrix.argtypes = [ctypes.c_int, vp, vp]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_get_threads.restype = ctypes.c_int
        L.or_mc_samples.argtypes = [i64, d, d]
        L.or_mc_samples.restype = i64
        _lib = L
    return _lib


def _f64(a, n=None):
    if a is None:
        return np.zeros(max(n or 1, 1), dtype=np.float64)
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prm(prm):
    a = np.zeros(8, dtype=np.float64)
    a[: len(prm)] = prm
    return a


def _nin(p_lo):
    return 0 if p_lo is None else int(np.asarray(p_lo).size)


def set_threads(n: int) -> None:
    """OpenMP threads for the oracle's loops started from the calling thread."""
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def uniform(seed: int, s: int, j: int, bits: int = 53) -> float:
    return lib().or_uniform(seed, s, j, bits)


def rhs(kind, prm, x, p=None, xh=None, ph=None, use_f=False, n_total=None, g0=0):
    """d(x, p, xh, ph) (or f(x, p) with use_f) evaluated at every cell."""
    x = _f64(x)
    n = x.size
    xh = x if xh is None else _f64(xh)
    n_in = _nin(p)
    p = _f64(p)
    ph = p if ph is None else _f64(ph)
    out = np.empty(n, dtype=np.float64)
    pr = _prm(prm)
    lib().or_rhs(kind, _p(pr), n if n_total is None else n_total, g0, n, n_in,
                 _p(x), _p(p), _p(xh), _p(ph), 1 if use_f else 0, _p(out))
    return out


def embed_rk4(kind, prm, x_lo, x_hi, p_lo=None, p_hi=None, t0=0.0, dt=0.01, nsteps=1,
              n_total=None, g0=0, n_in=None):
    """Algorithm 3: RK4 of the embedding system from (x_lo, x_hi).

    Works on the window [g0, g0+len) of an n_total-cell chain (default: the
    whole chain).  Returns (r_lo, r_hi) as float64 arrays.
    """
    x_lo, x_hi = _f64(x_lo), _f64(x_hi)
    length = x_lo.size
    if n_in is None:
        n_in = _nin(p_lo)
    pl, ph = _f64(p_lo), _f64(p_hi if p_hi is not None else p_lo)
    r_lo = np.empty(length, dtype=np.float64)
    r_hi = np.empty(length, dtype=np.float64)
    pr = _prm(prm)
    rc = lib().or_embed_rk4(kind, _p(pr), length if n_total is None else n_total, g0, length,
                            n_in, _p(x_lo), _p(x_hi), _p(pl), _p(ph), t0, dt, nsteps,
                            _p(r_lo), _p(r_hi))
    if rc != 0:
        raise RuntimeError(f"or_embed_rk4 failed ({rc})")
    return r_lo, r_hi


# ------------------------------------------------ user decomposition --
# A chain system given as C source text defining
#     REACH_DEVICE real reach_d(real xm, real x, real xp, real hm, real h, real hp,
#                               real u, real uh, const real* prm, long long i, long long n)
# (the same text the GPU library compiles with hipRTC).  Here it is compiled by
# the host C compiler with real = double and called by the oracle's own RK4.
USER_PRELUDE = "typedef double real;\n#define REACH_DEVICE static\n#include <math.h>\n"
USER_EXPORT = """
double or_user_entry(double xm, double x, double xp, double hm, double h, double hp,
                     double u, double uh, const double* prm, long long i, long long n)
{
    return reach_d(xm, x, xp, hm, h, hp, u, uh, prm, i, n);
}
"""


class UserSystem:
    """A user decomposition function compiled for the oracle."""

    def __init__(self, source: str):
        import hashlib
        import tempfile
        key = hashlib.sha256(source.encode()).hexdigest()[:16]
        d = os.path.join(tempfile.gettempdir(), "reach_oracle_user")
        os.makedirs(d, exist_ok=True)
        so = os.path.join(d, f"user_{key}.so")
        if not os.path.exists(so):
            c = os.path.join(d, f"user_{key}.c")
            with open(c, "w") as f:
                f.write(USER_PRELUDE + source + USER_EXPORT)
            subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                                   "-fno-fast-math", "-std=gnu99", c, "-o", so + ".tmp", "-lm"])
            os.replace(so + ".tmp", so)
        self.lib = ctypes.CDLL(so)
        self.fn = ctypes.cast(self.lib.or_user_entry, ctypes.c_void_p)


def embed_rk4_user(user: UserSystem, prm, x_lo, x_hi, p_lo=None, p_hi=None, dt=0.01,
                   nsteps=1, n_total=None, g0=0):
    """Algorithm 3 for a chain given by a user decomposition function."""
    x_lo, x_hi = _f64(x_lo), _f64(x_hi)
    length = x_lo.size
    n_in = _nin(p_lo)
    pl, ph = _f64(p_lo), _f64(p_hi if p_hi is not None else p_lo)
    r_lo = np.empty(length, dtype=np.float64)
    r_hi = np.empty(length, dtype=np.float64)
    pr = _prm(prm)
    rc = lib().or_embed_rk4_user(user.fn, _p(pr), length if n_total is None else n_total, g0,
                                 length, n_in, _p(x_lo), _p(x_hi), _p(pl), _p(ph), dt, nsteps,
                                 _p(r_lo), _p(r_hi))
    if rc != 0:
        raise RuntimeError(f"or_embed_rk4_user failed ({rc})")
    return r_lo, r_hi


def f_rk4_user(user: UserSystem, prm, x0, p=None, dt=0.01, nsteps=1):
    """RK4 of x' = d(x, p, x, p) from x0 (one trajectory)."""
    x0 = _f64(x0)
    n_in = _nin(p)
    pp = _f64(p)
    out = np.empty(x0.size, dtype=np.float64)
    pr = _prm(prm)
    rc = lib().or_f_rk4_user(user.fn, _p(pr), x0.size, n_in, _p(x0), _p(pp), dt, nsteps, _p(out))
    if rc != 0:
        raise RuntimeError(f"or_f_rk4_user failed ({rc})")
    return out


def montecarlo_user(user: UserSystem, prm, x_lo, x_hi, p_lo=None, p_hi=None, dt=0.01,
                    nsteps=1, m=1, seed=0, s0=0, ubits=53, return_samples=False):
    """Algorithm 4 for a user system over samples s0 .. s0+m-1."""
    x_lo, x_hi = _f64(x_lo), _f64(x_hi)
    n = x_lo.size
    n_in = _nin(p_lo)
    pl, ph = _f64(p_lo), _f64(p_hi if p_hi is not None else p_lo)
    r_min = np.empty(n, dtype=np.float64)
    r_max = np.empty(n, dtype=np.float64)
    samples = np.empty((m, n), dtype=np.float64) if return_samples else None
    pr = _prm(prm)
    rc = lib().or_montecarlo_user(user.fn, _p(pr), n, n_in, _p(x_lo), _p(x_hi), _p(pl), _p(ph),
                                  dt, nsteps, s0, m, seed, ubits, _p(r_min), _p(r_max),
                                  _p(samples))
    if rc != 0:
        raise RuntimeError(f"or_montecarlo_user failed ({rc})")
    if return_samples:
        return r_min, r_max, samples
    return r_min, r_max


def heat3d_prm(nx, ny, nz, alpha, dx):
    """Parameters of the 3-D heat system: grid extents, diffusivity, spacing."""
    return [float(nx), float(ny), float(nz), float(alpha), float(dx)]


def embed_rk4_grid(prm, x_lo, x_hi, org, dim, dt=0.01, nsteps=1):
    """Algorithm 3 on the window box [org, org + dim) of a 3-D heat grid.

    x_lo / x_hi hold the window's cells (x fastest).  Cells farther than
    4 nsteps from every cut face are bitwise those of a whole-grid run.
    """
    x_lo, x_hi = _f64(x_lo), _f64(x_hi)
    o = np.asarray(org, dtype=np.int64)
    dm = np.asarray(dim, dtype=np.int64)
    length = int(np.prod(dm))
    assert x_lo.size == length and x_hi.size == length
    r_lo = np.empty(length, dtype=np.float64)
    r_hi = np.empty(length, dtype=np.float64)
    pr = _prm(prm)
    rc = lib().or_embed_rk4_grid(_p(pr), _p(o), _p(dm), _p(x_lo), _p(x_hi), dt, nsteps,
                                 _p(r_lo), _p(r_hi))
    if rc != 0:
        raise RuntimeError(f"or_embed_rk4_grid failed ({rc})")
    return r_lo, r_hi


def heat3d_window(prm, box_fn, a, b, nsteps, dt=0.01):
    """Output cells of the box [a, b) (per-axis (x, y, z) bounds) of a
    whole-grid 3-D heat embedding run, from the light cone.

    ``box_fn(org, dim)`` returns the input cells (lo, hi) of the box
    [org, org + dim), x fastest.  Returns (r_lo, r_hi) of shape (z, y, x).
    """
    G = [int(prm[0]), int(prm[1]), int(prm[2])]
    r = 4 * nsteps
    org = [max(0, a[d] - r) for d in range(3)]
    end = [min(G[d], b[d] + r) for d in range(3)]
    dim = [end[d] - org[d] for d in range(3)]
    x_lo, x_hi = box_fn(org, dim)
    r_lo, r_hi = embed_rk4_grid(prm, x_lo, x_hi, org, dim, dt, nsteps)
    sl = tuple(slice(a[d] - org[d], b[d] - org[d]) for d in (2, 1, 0))
    shp = (dim[2], dim[1], dim[0])
    return r_lo.reshape(shp)[sl], r_hi.reshape(shp)[sl]


def f_rk4(kind, prm, x0, p=None, t0=0.0, dt=0.01, nsteps=1):
    """Classical RK4 of x' = f(x, p) from x0 (one trajectory)."""
    x0 = _f64(x0)
    n_in = _nin(p)
    pp = _f64(p)
    out = np.empty(x0.size, dtype=np.float64)
    pr = _prm(prm)
    rc = lib().or_f_rk4(kind, _p(pr), x0.size, n_in, _p(x0), _p(pp), t0, dt, nsteps, _p(out))
    if rc != 0:
        raise RuntimeError(f"or_f_rk4 failed ({rc})")
    return out


def montecarlo(kind, prm, x_lo, x_hi, p_lo=None, p_hi=None, t0=0.0, dt=0.01, nsteps=1,
               m=1, seed=0, s0=0, ubits=53, return_samples=False):
    """Algorithm 4 over samples s0 .. s0+m-1; returns (r_min, r_max[, samples])."""
    x_lo, x_hi = _f64(x_lo), _f64(x_hi)
    n = x_lo.size
    n_in = _nin(p_lo)
    pl, ph = _f64(p_lo), _f64(p_hi if p_hi is not None else p_lo)
    r_min = np.empty(n, dtype=np.float64)
    r_max = np.empty(n, dtype=np.float64)
    samples = np.empty((m, n), dtype=np.float64) if return_samples else None
    pr = _prm(prm)
    rc = lib().or_montecarlo(kind, _p(pr), n, n_in, _p(x_lo), _p(x_hi), _p(pl), _p(ph), t0, dt,
                             nsteps, s0, m, seed, ubits, _p(r_min), _p(r_max), _p(samples))
    if rc != 0:
        raise RuntimeError(f"or_montecarlo failed ({rc})")
    if return_samples:
        return r_min, r_max, samples
    return r_min, r_max


def growth_bound(kind, prm, x_lo, x_hi, p_lo=None, p_hi=None, t0=0.0, dt=0.01, nsteps=1,
                 n_total=None, g0=0):
    """Algorithm 2: contraction / growth-bound box; returns (r_lo, r_hi)."""
    x_lo, x_hi = _f64(x_lo), _f64(x_hi)
    length = x_lo.size
    n_in = _nin(p_lo)
    pl, ph = _f64(p_lo), _f64(p_hi if p_hi is not None else p_lo)
    r_lo = np.empty(length, dtype=np.float64)
    r_hi = np.empty(length, dtype=np.float64)
    pr = _prm(prm)
    rc = lib().or_growth_bound(kind, _p(pr), length if n_total is None else n_total, g0, length,
                               n_in, _p(x_lo), _p(x_hi), _p(pl), _p(ph), t0, dt, nsteps,
                               _p(r_lo), _p(r_hi))
    if rc != 0:
        raise RuntimeError(f"or_growth_bound failed ({rc})")
    return r_lo, r_hi


def contraction_matrix(kind, prm):
    """(sub, diag, super, input factor) of the tridiagonal contraction matrix."""
    pr = _prm(prm)
    out = np.zeros(4, dtype=np.float64)
    lib().or_contraction_matrix(kind, _p(pr), _p(out))
    return tuple(out)


def mc_samples(n: int, eps: float, delta: float) -> int:
    return int(lib().or_mc_samples(n, eps, delta))


def embed_window(kind, prm, box_fn, n_total, a, b, nsteps, p_lo=None, p_hi=None, t0=0.0,
                 dt=0.01):
    """Output cells [a, b) of a whole-chain embedding run, from the light cone.

    Each RK4 step lets a cell see 4 cells farther (one per stage), so cells
    [a, b) after nsteps steps depend only on input cells
    [a - 4 nsteps, b + 4 nsteps) clipped to the chain.  ``box_fn(i0, count)``
    returns those input cells (lo, hi).  The result is bitwise the whole-chain
    oracle's on [a, b).
    """
    r = 4 * nsteps
    lo_i = max(0, a - r)
    hi_i = min(n_total, b + r)
    x_lo, x_hi = box_fn(lo_i, hi_i - lo_i)
    r_lo, r_hi = embed_rk4(kind, prm, x_lo, x_hi, p_lo, p_hi, t0, dt, nsteps,
                           n_total=n_total, g0=lo_i)
    return r_lo[a - lo_i: b - lo_i], r_hi[a - lo_i: b - lo_i]
