"""Python binding of libreach.so, the MI355X interval-reachability library.

Argument marshalling only: every function below forwards to the C entry point
of the same name in ``include/reach.h``; all arithmetic runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and streams.  There is
no CPU fallback: if the library is missing, importing the functions fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libreach.so")

# status codes (reach.h)
REACH_OK = 0
REACH_PENDING = 1
REACH_E_INVAL = -1
REACH_E_NOMEM = -2
REACH_E_DEVICE = -3
REACH_E_UNSUPPORTED = -4
REACH_E_NONFINITE = -5
REACH_E_ORDER = -6
REACH_E_CANCELLED = -7
REACH_E_BUSY = -8
REACH_E_TIMEOUT = -9
STATUS_NAMES = {0: "OK", 1: "PENDING", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_DEVICE",
                -4: "E_UNSUPPORTED", -5: "E_NONFINITE", -6: "E_ORDER", -7: "E_CANCELLED",
                -8: "E_BUSY", -9: "E_TIMEOUT"}

REACH_F64, REACH_F32 = 0, 1
REACH_CTM, REACH_RD, REACH_LIN3, REACH_HEAT3D, REACH_USER = 1, 2, 3, 4, 5


class ReachError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


class reach_system(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("bc", ctypes.c_int32), ("n", ctypes.c_int64),
                ("n_in", ctypes.c_int64), ("prm", ctypes.c_double * 8)]


class reach_query(ctypes.Structure):
    _fields_ = [("sys", reach_system), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("x_lo", ctypes.c_void_p), ("x_hi", ctypes.c_void_p), ("p_lo", ctypes.c_void_p),
                ("p_hi", ctypes.c_void_p), ("r_lo", ctypes.c_void_p), ("r_hi", ctypes.c_void_p),
                ("t0", ctypes.c_double), ("dt", ctypes.c_double), ("nsteps", ctypes.c_int64)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libreach.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc, gfx950); there is no fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, d, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                ctypes.c_double, ctypes.c_size_t)
    P = ctypes.POINTER
    sysp = P(reach_system)
    qp = P(reach_query)
    sigs = {
        "reach_ctx_create": ([ctypes.c_int, P(vp)], i32),
        "reach_ctx_destroy": ([vp], None),
        "reach_last_error": ([vp], ctypes.c_char_p),
        "reach_set_option": ([vp, ctypes.c_char_p, i64], i32),
        "reach_get_option": ([vp, ctypes.c_char_p], i64),
        "reach_workspace_bytes": ([vp, sysp, i32, i64], sz),
        "reach_plan_embed": ([vp, sysp, i32, i64, P(i64)], i32),
        "reach_autotune_embed": ([vp, sysp, i32, vp, vp, vp, vp, d, i64, vp, vp, vp, sz, vp,
                                  P(i64)], i32),
        "reach_sync": ([vp, vp], i32),
        "reach_embed_rk4": ([vp, sysp, i32, vp, vp, vp, vp, d, d, i64, vp, vp, vp, sz, vp], i32),
        "reach_montecarlo": ([vp, sysp, i32, vp, vp, vp, vp, d, d, i64, i64, u64, vp, vp, vp, sz,
                              vp], i32),
        "reach_montecarlo_range": ([vp, sysp, i32, vp, vp, vp, vp, d, d, i64, i64, i64, u64, vp,
                                    vp, vp, sz, vp], i32),
        "reach_montecarlo_noalloc": ([vp, sysp, i32, vp, vp, vp, vp, d, d, i64, i64, i64, u64,
                                      vp, vp, vp], i32),
        "reach_noalloc_scratch_bytes": ([], sz),
        "reach_mc_samples": ([i64, d, d], i64),
        "reach_embed_rk4_tube": ([vp, sysp, i32, vp, vp, vp, vp, d, d, i64, i64, vp, vp, vp, sz,
                                  vp], i32),
        "reach_growth_bound_workspace_bytes": ([vp, sysp, i32], sz),
        "reach_growth_bound": ([vp, sysp, i32, vp, vp, vp, vp, d, d, i64, vp, vp, vp, sz, vp], i32),
        "reach_batch_workspace_bytes": ([i64], sz),
        "reach_embed_rk4_batch": ([vp, qp, i64, vp, sz, vp], i32),
        "reach_plan_batch": ([vp, qp, i64, P(i64), P(i32), P(i32), P(i64), P(i64)], i32),
        "reach_embed_rk4_each": ([vp, qp, i64, i32], i32),
        "reach_autotune_batch": ([vp, qp, i64, vp, sz, vp, P(i64)], i32),
        "reach_server_start": ([vp, vp, sz, i32, vp], i32),
        "reach_submit": ([vp, qp, P(u64)], i32),
        "reach_submit_at": ([vp, qp, d, P(u64)], i32),
        "reach_clock_us": ([], d),
        "reach_poll": ([vp, u64, P(i32)], i32),
        "reach_cancel": ([vp, u64], i32),
        "reach_server_stop": ([vp], i32),
        "reach_server_stats": ([vp, P(d), P(d), P(d), P(i64)], i32),
        "reach_user_create": ([vp, ctypes.c_char_p, P(vp)], i32),
        "reach_user_destroy": ([vp], None),
        "reach_embed_rk4_user": ([vp, vp, sysp, i32, vp, vp, vp, vp, d, d, i64, vp, vp, vp, sz,
                                  vp], i32),
        "reach_user_workspace_bytes": ([vp, sysp, i32, i64], sz),
        "reach_montecarlo_user": ([vp, vp, sysp, i32, vp, vp, vp, vp, d, d, i64, i64, i64, u64,
                                   vp, vp, vp, sz, vp], i32),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


_probe = None


def probe_lib():
    """libreach_probe.so: the HBM stream probe of the benchmark (reach_probe.h)."""
    global _probe
    if _probe is None:
        path = os.path.join(os.path.dirname(LIB_PATH), "libreach_probe.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(path)
        L.reach_probe_stream2.argtypes = [ctypes.c_void_p] * 4 + [
            ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p]
        L.reach_probe_stream2.restype = ctypes.c_int
        _probe = L
    return _probe


# --------------------------------------------------------------- helpers

def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr()
    return int(t)


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def steps_between(t0: float, t1: float, dt: float) -> int:
    """RK4 steps from t0 to t1 with step dt: round((t1 - t0) / dt), rejecting a
    horizon that is not a whole number of steps (mismatch above 1e-9 |t1 - t0|)."""
    span = float(t1) - float(t0)
    if not (dt > 0) or span < 0:
        raise ValueError("need dt > 0 and t1 >= t0")
    n = int(round(span / dt))
    if abs(n * dt - span) > 1e-9 * abs(span):
        raise ValueError(f"[t0, t1] = [{t0}, {t1}] is not a whole number of steps of {dt}")
    return n


def _nsteps(nsteps, t0, t1, dt) -> int:
    if t1 is None:
        if nsteps is None:
            raise ValueError("give nsteps or t1")
        return int(nsteps)
    n = steps_between(t0, t1, dt)
    if nsteps is not None and int(nsteps) != n:
        raise ValueError(f"nsteps = {nsteps} disagrees with t1 ({n} steps)")
    return n


def make_system(kind: int, n: int, prm, n_in: int = 0, bc: int = 0) -> reach_system:
    s = reach_system()
    s.kind = int(kind)
    s.bc = int(bc)
    s.n = int(n)
    s.n_in = int(n_in)
    for i, v in enumerate(prm):
        s.prm[i] = float(v)
    return s


def dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float64:
        return REACH_F64
    if dt == torch.float32:
        return REACH_F32
    raise ValueError(f"unsupported dtype {dt}")


def _check_tensor(t, name, dtype, n, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need contiguous {dtype} of {n} elements")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


# ------------------------------------------------------------ C-ABI names

def reach_ctx_create(device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = lib().reach_ctx_create(int(device), ctypes.byref(h))
    if st != REACH_OK:
        raise ReachError(st, f"reach_ctx_create(device={device})")
    return h


def reach_ctx_destroy(ctx) -> None:
    lib().reach_ctx_destroy(ctx)


def reach_last_error(ctx) -> str:
    v = lib().reach_last_error(ctx)
    return v.decode() if v else ""


def _chk(ctx, st, what):
    if st < 0:
        raise ReachError(st, f"{what}: {reach_last_error(ctx)}")
    return st


def reach_set_option(ctx, key: str, value: int) -> None:
    _chk(ctx, lib().reach_set_option(ctx, key.encode(), int(value)), "reach_set_option")


def reach_get_option(ctx, key: str) -> int:
    return int(lib().reach_get_option(ctx, key.encode()))


def reach_workspace_bytes(ctx, sys: reach_system, dtype: int, m: int = 0) -> int:
    v = lib().reach_workspace_bytes(ctx, ctypes.byref(sys), int(dtype), int(m))
    if v == ctypes.c_size_t(-1).value:
        raise ReachError(REACH_E_INVAL, f"reach_workspace_bytes: {reach_last_error(ctx)}")
    return int(v)


def reach_plan_embed(ctx, sys: reach_system, dtype: int, nsteps: int) -> dict:
    out = (ctypes.c_int64 * 7)()
    _chk(ctx, lib().reach_plan_embed(ctx, ctypes.byref(sys), int(dtype), int(nsteps), out),
         "reach_plan_embed")
    return dict(E=out[0], K=out[1], tiles=out[2], stride=out[3], halo=out[4], passes=out[5],
                S=out[6])


def reach_autotune_embed(ctx, sys: reach_system, dtype: int, x_lo, x_hi, p_lo, p_hi, dt: float,
                         trial_steps: int, r_lo, r_hi, workspace=None, workspace_bytes: int = 0,
                         stream=None) -> dict:
    out = (ctypes.c_int64 * 4)()
    _chk(ctx, lib().reach_autotune_embed(ctx, ctypes.byref(sys), int(dtype), _ptr(x_lo),
                                         _ptr(x_hi), _ptr(p_lo), _ptr(p_hi), float(dt),
                                         int(trial_steps), _ptr(r_lo), _ptr(r_hi),
                                         _ptr(workspace), int(workspace_bytes), _stream(stream),
                                         out), "reach_autotune_embed")
    return dict(E=out[0], K=out[1], fs_per_state_step=out[2], S=out[3])


def reach_sync(ctx, stream=None) -> int:
    """Returns the status code (REACH_OK, REACH_E_NONFINITE, REACH_E_ORDER...)."""
    return int(lib().reach_sync(ctx, _stream(stream)))


def reach_embed_rk4(ctx, sys: reach_system, dtype: int, x_lo, x_hi, p_lo, p_hi, t0: float,
                    dt: float, nsteps: int, r_lo, r_hi, workspace=None, workspace_bytes: int = 0,
                    stream=None) -> int:
    st = lib().reach_embed_rk4(ctx, ctypes.byref(sys), int(dtype), _ptr(x_lo), _ptr(x_hi),
                               _ptr(p_lo), _ptr(p_hi), float(t0), float(dt), int(nsteps),
                               _ptr(r_lo), _ptr(r_hi), _ptr(workspace), int(workspace_bytes),
                               _stream(stream))
    return _chk(ctx, st, "reach_embed_rk4")


def reach_montecarlo(ctx, sys: reach_system, dtype: int, x_lo, x_hi, p_lo, p_hi, t0: float,
                     dt: float, nsteps: int, m: int, seed: int, r_min, r_max, workspace=None,
                     workspace_bytes: int = 0, stream=None) -> int:
    st = lib().reach_montecarlo(ctx, ctypes.byref(sys), int(dtype), _ptr(x_lo), _ptr(x_hi),
                                _ptr(p_lo), _ptr(p_hi), float(t0), float(dt), int(nsteps), int(m),
                                int(seed), _ptr(r_min), _ptr(r_max), _ptr(workspace),
                                int(workspace_bytes), _stream(stream))
    return _chk(ctx, st, "reach_montecarlo")


def reach_montecarlo_range(ctx, sys: reach_system, dtype: int, x_lo, x_hi, p_lo, p_hi,
                           t0: float, dt: float, nsteps: int, s0: int, m: int, seed: int, r_min,
                           r_max, workspace=None, workspace_bytes: int = 0, stream=None) -> int:
    st = lib().reach_montecarlo_range(ctx, ctypes.byref(sys), int(dtype), _ptr(x_lo), _ptr(x_hi),
                                      _ptr(p_lo), _ptr(p_hi), float(t0), float(dt), int(nsteps),
                                      int(s0), int(m), int(seed), _ptr(r_min), _ptr(r_max),
                                      _ptr(workspace), int(workspace_bytes), _stream(stream))
    return _chk(ctx, st, "reach_montecarlo_range")


def reach_montecarlo_noalloc(ctx, sys: reach_system, dtype: int, x_lo, x_hi, p_lo, p_hi,
                             t0: float, dt: float, nsteps: int, s0: int, m: int, seed: int,
                             r_min, r_max, stream=None) -> int:
    st = lib().reach_montecarlo_noalloc(ctx, ctypes.byref(sys), int(dtype), _ptr(x_lo),
                                        _ptr(x_hi), _ptr(p_lo), _ptr(p_hi), float(t0), float(dt),
                                        int(nsteps), int(s0), int(m), int(seed), _ptr(r_min),
                                        _ptr(r_max), _stream(stream))
    return _chk(ctx, st, "reach_montecarlo_noalloc")


def reach_noalloc_scratch_bytes() -> int:
    return int(lib().reach_noalloc_scratch_bytes())


def reach_embed_rk4_tube(ctx, sys: reach_system, dtype: int, x_lo, x_hi, p_lo, p_hi, t0: float,
                         dt: float, nsteps: int, every: int, tube_lo, tube_hi, workspace=None,
                         workspace_bytes: int = 0, stream=None) -> int:
    st = lib().reach_embed_rk4_tube(ctx, ctypes.byref(sys), int(dtype), _ptr(x_lo), _ptr(x_hi),
                                    _ptr(p_lo), _ptr(p_hi), float(t0), float(dt), int(nsteps),
                                    int(every), _ptr(tube_lo), _ptr(tube_hi), _ptr(workspace),
                                    int(workspace_bytes), _stream(stream))
    return _chk(ctx, st, "reach_embed_rk4_tube")


def reach_growth_bound_workspace_bytes(ctx, sys: reach_system, dtype: int) -> int:
    v = lib().reach_growth_bound_workspace_bytes(ctx, ctypes.byref(sys), int(dtype))
    if v == ctypes.c_size_t(-1).value:
        raise ReachError(REACH_E_INVAL, f"reach_growth_bound_workspace_bytes: {reach_last_error(ctx)}")
    return int(v)


def reach_growth_bound(ctx, sys: reach_system, dtype: int, x_lo, x_hi, p_lo, p_hi, t0: float,
                       dt: float, nsteps: int, r_lo, r_hi, workspace=None, workspace_bytes: int = 0,
                       stream=None) -> int:
    st = lib().reach_growth_bound(ctx, ctypes.byref(sys), int(dtype), _ptr(x_lo), _ptr(x_hi),
                                  _ptr(p_lo), _ptr(p_hi), float(t0), float(dt), int(nsteps),
                                  _ptr(r_lo), _ptr(r_hi), _ptr(workspace), int(workspace_bytes),
                                  _stream(stream))
    return _chk(ctx, st, "reach_growth_bound")


def reach_user_create(ctx, source: str):
    """Compile a user decomposition function (C source text) for the context's
    device; returns the handle (free it with reach_user_destroy)."""
    h = ctypes.c_void_p()
    st = lib().reach_user_create(ctx, source.encode(), ctypes.byref(h))
    _chk(ctx, st, "reach_user_create")
    return h


def reach_user_destroy(user) -> None:
    lib().reach_user_destroy(user)


def reach_embed_rk4_user(ctx, user, sys: reach_system, dtype: int, x_lo, x_hi, p_lo, p_hi,
                         t0: float, dt: float, nsteps: int, r_lo, r_hi, workspace=None,
                         workspace_bytes: int = 0, stream=None) -> int:
    st = lib().reach_embed_rk4_user(ctx, user, ctypes.byref(sys), int(dtype), _ptr(x_lo),
                                    _ptr(x_hi), _ptr(p_lo), _ptr(p_hi), float(t0), float(dt),
                                    int(nsteps), _ptr(r_lo), _ptr(r_hi), _ptr(workspace),
                                    int(workspace_bytes), _stream(stream))
    return _chk(ctx, st, "reach_embed_rk4_user")


def reach_user_workspace_bytes(ctx, sys: reach_system, dtype: int, m: int) -> int:
    v = lib().reach_user_workspace_bytes(ctx, ctypes.byref(sys), int(dtype), int(m))
    if v == ctypes.c_size_t(-1).value:
        raise ReachError(REACH_E_INVAL, f"reach_user_workspace_bytes: {reach_last_error(ctx)}")
    return int(v)


def reach_montecarlo_user(ctx, user, sys: reach_system, dtype: int, x_lo, x_hi, p_lo, p_hi,
                          t0: float, dt: float, nsteps: int, s0: int, m: int, seed: int, r_min,
                          r_max, workspace=None, workspace_bytes: int = 0, stream=None) -> int:
    st = lib().reach_montecarlo_user(ctx, user, ctypes.byref(sys), int(dtype), _ptr(x_lo),
                                     _ptr(x_hi), _ptr(p_lo), _ptr(p_hi), float(t0), float(dt),
                                     int(nsteps), int(s0), int(m), int(seed), _ptr(r_min),
                                     _ptr(r_max), _ptr(workspace), int(workspace_bytes),
                                     _stream(stream))
    return _chk(ctx, st, "reach_montecarlo_user")


def reach_mc_samples(n: int, eps: float, delta: float) -> int:
    return int(lib().reach_mc_samples(int(n), float(eps), float(delta)))


def reach_batch_workspace_bytes(nq: int) -> int:
    return int(lib().reach_batch_workspace_bytes(int(nq)))


def reach_plan_batch(ctx, queries, with_E: bool = False) -> list:
    """The batch's work items in launch order, each a list of query indices
    (more than one: a segment pack sharing a wavefront); with_E: (E, list)
    pairs, E the pack's cells per lane (0: one query over the whole wave).
    Host only; ctx may be None."""
    arr = query_array(queries)
    nq = len(queries)
    start = (ctypes.c_int64 * max(nq, 1))()
    count = (ctypes.c_int32 * max(nq, 1))()
    ecnt = (ctypes.c_int32 * max(nq, 1))()
    member = (ctypes.c_int64 * max(nq, 1))()
    ni = ctypes.c_int64(0)
    st = lib().reach_plan_batch(ctx, arr, nq, start, count, ecnt, member, ctypes.byref(ni))
    if ctx is None:
        if st != REACH_OK:
            raise ReachError(st, "reach_plan_batch")
    else:
        _chk(ctx, st, "reach_plan_batch")
    items = [[int(member[start[k] + m]) for m in range(count[k])] for k in range(ni.value)]
    if with_E:
        return [(int(ecnt[k]), items[k]) for k in range(ni.value)]
    return items


def query_array(queries):
    """A ctypes array of reach_query (build once, pass to the batch calls)."""
    if isinstance(queries, ctypes.Array):
        return queries
    return (reach_query * len(queries))(*queries)


def reach_embed_rk4_batch(ctx, queries, workspace, workspace_bytes: int, stream=None) -> int:
    arr = query_array(queries)
    st = lib().reach_embed_rk4_batch(ctx, arr, len(queries), _ptr(workspace),
                                     int(workspace_bytes), _stream(stream))
    return _chk(ctx, st, "reach_embed_rk4_batch")


def reach_autotune_batch(ctx, queries, workspace, workspace_bytes: int, stream=None) -> dict:
    arr = query_array(queries)
    best = (ctypes.c_int64 * 2)()
    st = lib().reach_autotune_batch(ctx, arr, len(queries), _ptr(workspace), int(workspace_bytes),
                                    _stream(stream), best)
    _chk(ctx, st, "reach_autotune_batch")
    return {"waves": int(best[0]), "batch_ns": int(best[1])}


def reach_embed_rk4_each(ctx, queries, nstreams: int = 8) -> int:
    arr = query_array(queries)
    st = lib().reach_embed_rk4_each(ctx, arr, len(queries), int(nstreams))
    return _chk(ctx, st, "reach_embed_rk4_each")


def reach_server_start(ctx, pool, pool_bytes: int, max_slots: int, stream=0) -> int:
    st = lib().reach_server_start(ctx, _ptr(pool), int(pool_bytes), int(max_slots),
                                  None if not stream else _stream(stream))
    return _chk(ctx, st, "reach_server_start")


def reach_submit(ctx, q: reach_query) -> int:
    t = ctypes.c_uint64()
    st = lib().reach_submit(ctx, ctypes.byref(q), ctypes.byref(t))
    _chk(ctx, st, "reach_submit")
    return int(t.value)


def reach_submit_at(ctx, q: reach_query, arrival_us: float) -> int:
    t = ctypes.c_uint64()
    st = lib().reach_submit_at(ctx, ctypes.byref(q), float(arrival_us), ctypes.byref(t))
    _chk(ctx, st, "reach_submit_at")
    return int(t.value)


def reach_clock_us() -> float:
    return float(lib().reach_clock_us())


def reach_poll(ctx, ticket: int):
    """(status of the call, final status of the query or None while pending)."""
    r = ctypes.c_int32(0)
    st = lib().reach_poll(ctx, int(ticket), ctypes.byref(r))
    if st == REACH_PENDING:
        return st, None
    _chk(ctx, st, "reach_poll")
    return st, int(r.value)


def reach_cancel(ctx, ticket: int) -> int:
    return int(lib().reach_cancel(ctx, int(ticket)))


def reach_server_stop(ctx) -> int:
    return _chk(ctx, lib().reach_server_stop(ctx), "reach_server_stop")


def reach_server_stats(ctx):
    p50, p99, mx = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    cnt = ctypes.c_int64()
    _chk(ctx, lib().reach_server_stats(ctx, ctypes.byref(p50), ctypes.byref(p99),
                                       ctypes.byref(mx), ctypes.byref(cnt)),
         "reach_server_stats")
    return dict(p50_us=p50.value, p99_us=p99.value, max_us=mx.value, completed=cnt.value)


# ------------------------------------------------------------ conveniences

def make_query(kind, n, prm, dtype_code_, x_lo, x_hi, r_lo, r_hi, dt, nsteps, p_lo=None,
               p_hi=None, t0=0.0, n_in=0) -> reach_query:
    """A reach_query; array arguments are tensors (device) or raw addresses."""
    q = reach_query()
    q.sys = make_system(kind, n, prm, n_in)
    q.dtype = dtype_code_
    q.reserved = 0
    q.x_lo, q.x_hi = _ptr(x_lo), _ptr(x_hi)
    q.p_lo, q.p_hi = _ptr(p_lo), _ptr(p_hi)
    q.r_lo, q.r_hi = _ptr(r_lo), _ptr(r_hi)
    q.t0, q.dt, q.nsteps = float(t0), float(dt), int(nsteps)
    return q


class Reach:
    """A context plus workspace management around the C entry points."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        self.ctx = reach_ctx_create(device)
        self._ws = None

    def close(self):
        if self.ctx is not None:
            reach_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes: int) -> torch.Tensor | None:
        if nbytes == 0:
            return None
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def set_option(self, key, value):
        reach_set_option(self.ctx, key, value)

    def embed(self, kind, prm, x_lo, x_hi, dt, nsteps=None, p_lo=None, p_hi=None, t0=0.0,
              r_lo=None, r_hi=None, stream=None, t1=None):
        nsteps = _nsteps(nsteps, t0, t1, dt)
        n = x_lo.numel()
        n_in = 0 if p_lo is None else p_lo.numel()
        dtc = dtype_code(x_lo.dtype)
        for name, t in (("x_lo", x_lo), ("x_hi", x_hi)):
            _check_tensor(t, name, x_lo.dtype, n, x_lo.device)
        if p_lo is not None:
            _check_tensor(p_lo, "p_lo", x_lo.dtype, n_in, x_lo.device)
            _check_tensor(p_hi, "p_hi", x_lo.dtype, n_in, x_lo.device)
        if r_lo is None:
            r_lo = torch.empty_like(x_lo)
        if r_hi is None:
            r_hi = torch.empty_like(x_hi)
        sys = make_system(kind, n, prm, n_in)
        nb = reach_workspace_bytes(self.ctx, sys, dtc, 0)
        ws = self.workspace(nb)
        reach_embed_rk4(self.ctx, sys, dtc, x_lo, x_hi, p_lo, p_hi, t0, dt, nsteps, r_lo, r_hi,
                        ws, nb, stream)
        return r_lo, r_hi

    def montecarlo(self, kind, prm, x_lo, x_hi, dt, nsteps, m, seed, p_lo=None, p_hi=None,
                   t0=0.0, s0=0, r_min=None, r_max=None, stream=None, t1=None):
        nsteps = _nsteps(nsteps, t0, t1, dt)
        n = x_lo.numel()
        n_in = 0 if p_lo is None else p_lo.numel()
        dtc = dtype_code(x_lo.dtype)
        _check_tensor(x_lo, "x_lo", x_lo.dtype, n, x_lo.device)
        _check_tensor(x_hi, "x_hi", x_lo.dtype, n, x_lo.device)
        if r_min is None:
            r_min = torch.empty_like(x_lo)
        if r_max is None:
            r_max = torch.empty_like(x_lo)
        sys = make_system(kind, n, prm, n_in)
        nb = reach_workspace_bytes(self.ctx, sys, dtc, m)
        ws = self.workspace(nb)
        reach_montecarlo_range(self.ctx, sys, dtc, x_lo, x_hi, p_lo, p_hi, t0, dt, nsteps, s0, m,
                               seed, r_min, r_max, ws, nb, stream)
        return r_min, r_max

    def user(self, source: str):
        """Compile a user decomposition function; returns its handle."""
        return reach_user_create(self.ctx, source)

    def embed_user(self, user, prm, x_lo, x_hi, dt, nsteps=None, p_lo=None, p_hi=None, t0=0.0,
                   r_lo=None, r_hi=None, stream=None, t1=None):
        nsteps = _nsteps(nsteps, t0, t1, dt)
        n = x_lo.numel()
        n_in = 0 if p_lo is None else p_lo.numel()
        dtc = dtype_code(x_lo.dtype)
        _check_tensor(x_lo, "x_lo", x_lo.dtype, n, x_lo.device)
        _check_tensor(x_hi, "x_hi", x_lo.dtype, n, x_lo.device)
        if p_lo is not None:
            _check_tensor(p_lo, "p_lo", x_lo.dtype, n_in, x_lo.device)
            _check_tensor(p_hi, "p_hi", x_lo.dtype, n_in, x_lo.device)
        if r_lo is None:
            r_lo = torch.empty_like(x_lo)
        if r_hi is None:
            r_hi = torch.empty_like(x_hi)
        sys = make_system(REACH_USER, n, prm, n_in)
        nb = 2 * n * x_lo.element_size()
        ws = self.workspace(nb)
        reach_embed_rk4_user(self.ctx, user, sys, dtc, x_lo, x_hi, p_lo, p_hi, t0, dt, nsteps,
                             r_lo, r_hi, ws, nb, stream)
        return r_lo, r_hi

    def montecarlo_user(self, user, prm, x_lo, x_hi, dt, nsteps, m, seed, p_lo=None, p_hi=None,
                        t0=0.0, s0=0, r_min=None, r_max=None, stream=None, t1=None):
        nsteps = _nsteps(nsteps, t0, t1, dt)
        n = x_lo.numel()
        n_in = 0 if p_lo is None else p_lo.numel()
        dtc = dtype_code(x_lo.dtype)
        _check_tensor(x_lo, "x_lo", x_lo.dtype, n, x_lo.device)
        _check_tensor(x_hi, "x_hi", x_lo.dtype, n, x_lo.device)
        if r_min is None:
            r_min = torch.empty_like(x_lo)
        if r_max is None:
            r_max = torch.empty_like(x_lo)
        sys = make_system(REACH_USER, n, prm, n_in)
        nb = reach_user_workspace_bytes(self.ctx, sys, dtc, m)
        ws = self.workspace(nb)
        reach_montecarlo_user(self.ctx, user, sys, dtc, x_lo, x_hi, p_lo, p_hi, t0, dt, nsteps,
                              s0, m, seed, r_min, r_max, ws, nb, stream)
        return r_min, r_max

    def growth_bound(self, kind, prm, x_lo, x_hi, dt, nsteps=None, p_lo=None, p_hi=None, t0=0.0,
                     r_lo=None, r_hi=None, stream=None, t1=None):
        nsteps = _nsteps(nsteps, t0, t1, dt)
        n = x_lo.numel()
        n_in = 0 if p_lo is None else p_lo.numel()
        dtc = dtype_code(x_lo.dtype)
        _check_tensor(x_lo, "x_lo", x_lo.dtype, n, x_lo.device)
        _check_tensor(x_hi, "x_hi", x_lo.dtype, n, x_lo.device)
        if r_lo is None:
            r_lo = torch.empty_like(x_lo)
        if r_hi is None:
            r_hi = torch.empty_like(x_hi)
        sys = make_system(kind, n, prm, n_in)
        nb = reach_growth_bound_workspace_bytes(self.ctx, sys, dtc)
        ws = self.workspace(nb)
        reach_growth_bound(self.ctx, sys, dtc, x_lo, x_hi, p_lo, p_hi, t0, dt, nsteps, r_lo, r_hi,
                           ws, nb, stream)
        return r_lo, r_hi

    def sync(self, stream=None) -> int:
        return reach_sync(self.ctx, stream)
