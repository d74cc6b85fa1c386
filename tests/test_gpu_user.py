"""GPU parity of user-defined chain systems (a decomposition function given
as C source text, compiled at run time with hipRTC) against the oracle's run
of the same text (Sec. 2.1 embedding, Algorithm 3 with the RK4 of
Algorithm 1)."""
import numpy as np
import pytest

import oracle
import workloads
from tests import user_sources as us
from tests.gpu_util import RTOL, assert_rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2001_10635_amd")

LIN3_COEF = (-0.5, -1.0, 0.75, -1.5)


@pytest.fixture(scope="module")
def rc():
    r = R.Reach(0)
    yield r
    r.close()


@pytest.fixture(scope="module")
def users(rc):
    out = {}
    for name in ("LIN3", "CTM", "RD", "SINE"):
        say(f"hipRTC compile of the {name} user source")
        out[name] = (rc.user(getattr(us, name)), oracle.UserSystem(getattr(us, name)))
    yield out
    for g, _ in out.values():
        R.reach_user_destroy(g)


@pytest.fixture(autouse=True)
def _reset(rc):
    rc.set_option("user.E", 0)
    rc.set_option("user.K", 0)
    yield
    rc.set_option("user.E", 0)
    rc.set_option("user.K", 0)


def sine_case(n, dtype, seed, inputs="scalar"):
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-3.0, 3.0, n)
    hi = lo + rng.uniform(0.0, 0.8, n)
    if inputs == "scalar":
        pl, ph = np.array([-0.2]), np.array([0.3])
    elif inputs == "cell":
        pl = rng.uniform(-0.3, 0.0, n)
        ph = pl + rng.uniform(0.0, 0.6, n)
    else:
        pl = ph = None
    c = lambda a: None if a is None else np.asarray(a).astype(dtype)
    return c(lo), c(hi), c(pl), c(ph)


def run_user(rc, g, prm, lo, hi, pl, ph, dt, nsteps):
    dev = lambda a: None if a is None else to_dev(a)
    r_lo, r_hi = rc.embed_user(g, prm, dev(lo), dev(hi), dt, nsteps, p_lo=dev(pl), p_hi=dev(ph))
    return to_host(r_lo), to_host(r_hi), rc.sync()


def oracle_user(o, prm, lo, hi, pl, ph, dt, nsteps):
    f = lambda a: None if a is None else np.asarray(a, dtype=np.float64)
    return oracle.embed_rk4_user(o, prm, f(lo), f(hi), f(pl), f(ph), dt=dt, nsteps=nsteps)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n", [1, 5, 64, 65, 511, 512, 513, 3001])
@pytest.mark.parametrize("inputs", ["none", "scalar", "cell"])
def test_user_sine_matches_oracle(rc, users, n, dtype, inputs):
    g, o = users["SINE"]
    lo, hi, pl, ph = sine_case(n, dtype, seed=n + 3, inputs=inputs)
    say(f"user sine n={n} {np.dtype(dtype).name} inputs={inputs}")
    g_lo, g_hi, st = run_user(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, 37)
    assert st == R.REACH_OK
    o_lo, o_hi = oracle_user(o, us.SINE_PRM, lo, hi, pl, ph, 0.05, 37)
    rt = RTOL[np.dtype(dtype)]
    assert_rel(g_lo, o_lo, rt, "lower")
    assert_rel(g_hi, o_hi, rt, "upper")


@pytest.mark.parametrize("E,K", [(1, 1), (2, 3), (4, 5), (8, 8), (8, 1), (1, 7)])
def test_user_multitile_matches_oracle_and_is_shape_invariant(rc, users, E, K):
    g, o = users["SINE"]
    n, nsteps = 3001, 29
    lo, hi, pl, ph = sine_case(n, np.float64, seed=61)
    rc.set_option("user.E", E)
    rc.set_option("user.K", K)
    say(f"user sine multitile E={E} K={K}")
    g_lo, g_hi, st = run_user(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, nsteps)
    assert st == R.REACH_OK
    o_lo, o_hi = oracle_user(o, us.SINE_PRM, lo, hi, pl, ph, 0.05, nsteps)
    assert_rel(g_lo, o_lo, 1e-12, "lower")
    assert_rel(g_hi, o_hi, 1e-12, "upper")
    rc.set_option("user.E", 0)
    rc.set_option("user.K", 0)
    d_lo, d_hi, _ = run_user(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, nsteps)
    assert np.array_equal(d_lo, g_lo) and np.array_equal(d_hi, g_hi)


@pytest.mark.parametrize("name", ["LIN3", "CTM", "RD"])
@pytest.mark.parametrize("n", [7, 700, 5000])
def test_user_restated_builtin_matches_builtin_and_oracle(rc, users, name, n):
    """The built-in systems restated as user text: the user kernel agrees with
    the built-in kernel and with the oracle."""
    g, o = users[name]
    rng = np.random.default_rng(n)
    if name == "LIN3":
        kind, prm, dt = R.REACH_LIN3, LIN3_COEF, 0.05
        lo = rng.uniform(-1, 1, n)
        hi = lo + rng.uniform(0, 0.5, n)
        pl = rng.uniform(-0.25, 0.0, n)
        ph = pl + rng.uniform(0.0, 0.5, n)
    elif name == "CTM":
        kind, prm, dt = R.REACH_CTM, workloads.CTM_PRM, 0.01
        lo, hi = workloads.box(workloads.CTM_RANDW, (12.0, 2.0), n, n)
        pl = ph = None
    else:
        kind, prm, dt = R.REACH_RD, (1.0,), 0.1
        lo, hi = workloads.box(workloads.SIN, (0.02,), n, n)
        pl, ph = np.array([-0.1]), np.array([0.1])
    say(f"user {name} n={n}")
    g_lo, g_hi, st = run_user(rc, g, prm, lo, hi, pl, ph, dt, 45)
    assert st == R.REACH_OK
    dev = lambda a: None if a is None else to_dev(a)
    b_lo, b_hi = rc.embed(kind, prm, dev(lo), dev(hi), dt, 45, p_lo=dev(pl), p_hi=dev(ph))
    assert rc.sync() == R.REACH_OK
    o_lo, o_hi = oracle_user(o, prm, lo, hi, pl, ph, dt, 45)
    assert_rel(g_lo, o_lo, 1e-12, "user vs oracle lower")
    assert_rel(g_hi, o_hi, 1e-12, "user vs oracle upper")
    assert_rel(g_lo, to_host(b_lo), 1e-12, "user vs built-in lower")
    assert_rel(g_hi, to_host(b_hi), 1e-12, "user vs built-in upper")


def test_user_resume_alias_and_zero_steps(rc, users):
    g, _ = users["SINE"]
    lo, hi, pl, ph = sine_case(4000, np.float64, seed=62)
    say("user resume / alias")
    a_lo, a_hi, _ = run_user(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, 20)
    b_lo, b_hi, _ = run_user(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, 8)
    c_lo, c_hi, _ = run_user(rc, g, us.SINE_PRM, b_lo, b_hi, pl, ph, 0.05, 12)
    assert np.array_equal(a_lo, c_lo) and np.array_equal(a_hi, c_hi)
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    rc.embed_user(g, us.SINE_PRM, x_lo, x_hi, 0.05, 20, p_lo=to_dev(pl), p_hi=to_dev(ph),
                  r_lo=x_lo, r_hi=x_hi)
    assert rc.sync() == R.REACH_OK
    assert np.array_equal(to_host(x_lo), a_lo) and np.array_equal(to_host(x_hi), a_hi)
    z_lo, z_hi, st = run_user(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, 0)
    assert st == R.REACH_OK and np.array_equal(z_lo, lo) and np.array_equal(z_hi, hi)


def test_user_errors(rc, users):
    say("user compile error")
    with pytest.raises(R.ReachError) as ei:
        rc.user("REACH_DEVICE real reach_d(real xm) { return undefined_name; }")
    assert ei.value.status == R.REACH_E_INVAL
    assert "undefined_name" in str(ei.value)          # the compiler's log is passed on
    g, _ = users["SINE"]
    x = to_dev(np.zeros(16))
    lib = R.lib()
    sys_user = R.make_system(R.REACH_USER, 16, us.SINE_PRM)
    st = lib.reach_embed_rk4(rc.ctx, R.ctypes.byref(sys_user), R.REACH_F64, x.data_ptr(),
                             x.data_ptr(), None, None, 0.0, 0.05, 1, x.data_ptr(), x.data_ptr(),
                             None, 0, None)
    assert st == R.REACH_E_INVAL
    sys_ctm = R.make_system(R.REACH_CTM, 16, workloads.CTM_PRM)
    st = lib.reach_embed_rk4_user(rc.ctx, g, R.ctypes.byref(sys_ctm), R.REACH_F64, x.data_ptr(),
                                  x.data_ptr(), None, None, 0.0, 0.05, 1, x.data_ptr(),
                                  x.data_ptr(), None, 0, None)
    assert st == R.REACH_E_INVAL
    st = lib.reach_embed_rk4_user(rc.ctx, None, R.ctypes.byref(sys_user), R.REACH_F64,
                                  x.data_ptr(), x.data_ptr(), None, None, 0.0, 0.05, 1,
                                  x.data_ptr(), x.data_ptr(), None, 0, None)
    assert st == R.REACH_E_INVAL
    with pytest.raises(R.ReachError):
        rc.set_option("user.E", 16)
        rc.embed_user(g, us.SINE_PRM, to_dev(np.zeros(4000)), to_dev(np.zeros(4000)), 0.05, 3)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("inputs", ["scalar", "cell"])
@pytest.mark.parametrize("n", [300, 5000])
def test_user_rd_in_builtin_order_equals_builtin_bitwise(rc, n, dtype, inputs):
    """Same per-cell arithmetic as the built-in RD kernel (and different tile
    shapes, halos and pass counts): identical results."""
    g = rc.user(us.RD_FUSED)
    try:
        rng = np.random.default_rng(n + 7)
        lo = rng.uniform(-1.0, 1.0, n).astype(dtype)
        hi = (lo + rng.uniform(0.0, 0.2, n)).astype(dtype)
        if inputs == "scalar":
            pl, ph = np.array([-0.1], dtype), np.array([0.1], dtype)
        else:
            pl = rng.uniform(-0.1, 0.0, n).astype(dtype)
            ph = (pl + rng.uniform(0.0, 0.2, n)).astype(dtype)
        say(f"user RD in built-in order n={n} {np.dtype(dtype).name} {inputs}")
        u_lo, u_hi, st = run_user(rc, g, (1.0, 2.0), lo, hi, pl, ph, 0.05, 41)
        assert st == R.REACH_OK
        b_lo, b_hi = rc.embed(R.REACH_RD, (1.0,), to_dev(lo), to_dev(hi), 0.05, 41,
                              p_lo=to_dev(pl), p_hi=to_dev(ph))
        assert rc.sync() == R.REACH_OK
        assert np.array_equal(u_lo, to_host(b_lo)) and np.array_equal(u_hi, to_host(b_hi))
    finally:
        R.reach_user_destroy(g)


# ------------------------------------------------------------ Monte Carlo

def oracle_user_mc(o, prm, lo, hi, pl, ph, dt, nsteps, m, seed, s0=0, ubits=53):
    f = lambda a: None if a is None else np.asarray(a, dtype=np.float64)
    return oracle.montecarlo_user(o, prm, f(lo), f(hi), f(pl), f(ph), dt=dt, nsteps=nsteps, m=m,
                                  seed=seed, s0=s0, ubits=ubits)


def run_user_mc(rc, g, prm, lo, hi, pl, ph, dt, nsteps, m, seed, s0=0):
    dev = lambda a: None if a is None else to_dev(a)
    mn, mx = rc.montecarlo_user(g, prm, dev(lo), dev(hi), dt, nsteps, m, seed, p_lo=dev(pl),
                                p_hi=dev(ph), s0=s0)
    return to_host(mn), to_host(mx), rc.sync()


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n", [1, 5, 64, 200, 512])
@pytest.mark.parametrize("inputs", ["none", "scalar", "cell"])
def test_user_mc_matches_oracle(rc, users, n, dtype, inputs):
    g, o = users["SINE"]
    lo, hi, pl, ph = sine_case(n, dtype, seed=n + 90, inputs=inputs)
    say(f"user mc sine n={n} {np.dtype(dtype).name} inputs={inputs}")
    g_mn, g_mx, st = run_user_mc(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, 25, 300, 17)
    assert st == R.REACH_OK
    ub = 53 if dtype == np.float64 else 24
    o_mn, o_mx = oracle_user_mc(o, us.SINE_PRM, lo, hi, pl, ph, 0.05, 25, 300, 17, ubits=ub)
    rt = RTOL[np.dtype(dtype)]
    assert_rel(g_mn, o_mn, rt, "min")
    assert_rel(g_mx, o_mx, rt, "max")


def test_user_mc_ranges_compose_and_sit_in_the_box(rc, users):
    g, _ = users["SINE"]
    lo, hi, pl, ph = sine_case(300, np.float64, seed=91)
    say("user mc ranges")
    a_mn, a_mx, _ = run_user_mc(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, 30, 500, 5)
    b_mn, b_mx, _ = run_user_mc(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, 30, 180, 5)
    c_mn, c_mx, _ = run_user_mc(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, 30, 320, 5, s0=180)
    assert np.array_equal(a_mn, np.minimum(b_mn, c_mn)) and np.array_equal(a_mx, np.maximum(b_mx, c_mx))
    e_lo, e_hi, _ = run_user(rc, g, us.SINE_PRM, lo, hi, pl, ph, 0.05, 30)
    assert np.all(a_mn >= e_lo - 1e-12) and np.all(a_mx <= e_hi + 1e-12)


def test_user_mc_restated_ctm_matches_builtin(rc, users):
    g, _ = users["CTM"]
    p = workloads.ctm64_f64()
    lo, hi = p.box()
    say("user mc ctm vs built-in")
    u_mn, u_mx, st = run_user_mc(rc, g, p.prm, lo, hi, None, None, p.dt, p.nsteps, 1000, p.seed)
    assert st == R.REACH_OK
    b_mn, b_mx = rc.montecarlo(p.kind, p.prm, to_dev(lo), to_dev(hi), p.dt, p.nsteps, 1000, p.seed)
    assert rc.sync() == R.REACH_OK
    assert_rel(u_mn, to_host(b_mn), 1e-12, "min")
    assert_rel(u_mx, to_host(b_mx), 1e-12, "max")


def test_user_mc_rejects_long_chains(rc, users):
    g, _ = users["SINE"]
    x = to_dev(np.zeros(600))
    sysd = R.make_system(R.REACH_USER, 600, us.SINE_PRM)
    st = R.lib().reach_montecarlo_user(rc.ctx, g, R.ctypes.byref(sysd), R.REACH_F64, x.data_ptr(),
                                       x.data_ptr(), None, None, 0.0, 0.05, 1, 0, 16, 1,
                                       x.data_ptr(), x.data_ptr(), x.data_ptr(), 1 << 20, None)
    assert st == R.REACH_E_UNSUPPORTED
