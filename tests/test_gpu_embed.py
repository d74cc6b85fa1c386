"""GPU parity of reach_embed_rk4 against the FP64 oracle (mixed monotonicity,
Sec. 2.1 / Algorithm 3 with the classical RK4 of Algorithm 1)."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import RTOL, assert_rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2001_10635_amd")

LIN3_COEF = (-0.5, -1.0, 0.75, -1.5)
VARIANTS = ["ctm", "rd", "rd_cell", "lin3", "lin3_cell"]
KIND = {"ctm": R.REACH_CTM, "rd": R.REACH_RD, "rd_cell": R.REACH_RD, "lin3": R.REACH_LIN3,
        "lin3_cell": R.REACH_LIN3}


@pytest.fixture(scope="module")
def rc():
    r = R.Reach(0)
    yield r
    r.close()


@pytest.fixture(autouse=True)
def _reset_options(rc):
    for k in ("embed.E", "embed.K", "embed.S"):
        rc.set_option(k, 0)
    yield
    for k in ("embed.E", "embed.K", "embed.S"):
        rc.set_option(k, 0)


def make_case(variant, n, dtype, seed):
    """(kind, prm, lo, hi, p_lo, p_hi, dt) as numpy arrays of `dtype`."""
    rng = np.random.default_rng(seed)
    kind = KIND[variant]
    pl = ph = None
    if variant == "ctm":
        lo, hi = workloads.box(workloads.CTM_RANDW, (12.0, 2.0), seed, n, dtype=dtype)
        prm, dt = workloads.CTM_PRM, 0.01
    elif variant.startswith("rd"):
        lo, hi = workloads.box(workloads.SIN, (0.02,), seed, n, dtype=dtype)
        prm, dt = (1.0,), 0.1
        if variant == "rd_cell":
            pl = rng.uniform(-0.1, 0.0, n)
            ph = pl + rng.uniform(0.0, 0.2, n)
        else:
            pl, ph = np.array([-0.1]), np.array([0.1])
    else:
        lo = rng.uniform(-1.0, 1.0, n)
        hi = lo + rng.uniform(0.0, 0.5, n)
        prm, dt = LIN3_COEF, 0.05
        if variant == "lin3_cell":
            pl = rng.uniform(-0.25, 0.0, n)
            ph = pl + rng.uniform(0.0, 0.5, n)
        else:
            pl, ph = np.array([-0.25]), np.array([0.5])
    cast = lambda a: None if a is None else np.asarray(a).astype(dtype)
    return kind, prm, cast(lo), cast(hi), cast(pl), cast(ph), dt


def run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, nsteps, **kw):
    dev = lambda a: None if a is None else to_dev(a)
    r_lo, r_hi = rc.embed(kind, prm, dev(lo), dev(hi), dt, nsteps, p_lo=dev(pl), p_hi=dev(ph), **kw)
    st = rc.sync()
    return to_host(r_lo), to_host(r_hi), st


def run_oracle(kind, prm, lo, hi, pl, ph, dt, nsteps):
    f = lambda a: None if a is None else np.asarray(a, dtype=np.float64)
    return oracle.embed_rk4(kind, prm, f(lo), f(hi), f(pl), f(ph), dt=dt, nsteps=nsteps)


SIZES = [1, 2, 3, 4, 5, 63, 64, 65, 127, 511, 512, 513, 1000, 2049, 4097]


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n", SIZES)
def test_embed_matches_oracle(rc, variant, n, dtype):
    case = make_case(variant, n, dtype, seed=1000 + n)
    nsteps = 37
    say(f"embed {variant} n={n} {np.dtype(dtype).name} N={nsteps}")
    g_lo, g_hi, st = run_gpu(rc, *case, nsteps)
    assert st == R.REACH_OK
    o_lo, o_hi = run_oracle(*case, nsteps)
    rt = RTOL[np.dtype(dtype)]
    assert_rel(g_lo, o_lo, rt, "lower")
    assert_rel(g_hi, o_hi, rt, "upper")


@pytest.mark.parametrize("E,K,S", [(1, 1, 2), (2, 3, 2), (4, 7, 2), (8, 8, 2), (16, 4, 2),
                                   (12, 5, 2), (1, 1, 1), (4, 3, 1), (8, 9, 1), (24, 11, 1),
                                   (28, 13, 1), (32, 6, 1)])
@pytest.mark.parametrize("variant", ["ctm", "rd", "rd_cell", "lin3", "lin3_cell"])
def test_multitile_halos_match_oracle(rc, variant, E, K, S):
    """Forced small tiles: many windows, cut edges, a masked last window."""
    if S == 1 and variant.startswith("lin3"):
        pytest.skip("the coupled LIN3 chain runs both sides per wave")
    n, nsteps = 3001, 29
    case = make_case(variant, n, np.float64, seed=77)
    rc.set_option("embed.S", S)
    rc.set_option("embed.E", E)
    rc.set_option("embed.K", K)
    say(f"multitile {variant} E={E} K={K} S={S}")
    g_lo, g_hi, st = run_gpu(rc, *case, nsteps)
    assert st == R.REACH_OK
    o_lo, o_hi = run_oracle(*case, nsteps)
    assert_rel(g_lo, o_lo, 1e-12, "lower")
    assert_rel(g_hi, o_hi, 1e-12, "upper")


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("variant", ["ctm", "rd"])
def test_tile_shape_invariance_is_bitwise(rc, variant, dtype):
    """Per-cell arithmetic does not depend on the tile shape or steps per pass."""
    n, nsteps = 20011, 41
    case = make_case(variant, n, dtype, seed=5)
    outs = []
    shapes = [(2, 1, 2), (4, 3, 2), (8, 8, 2), (12, 12, 2), (16, 8, 2), (8, 1, 1), (16, 10, 1),
              (24, 12, 1), (32, 16, 1)]
    if dtype == np.float32:
        shapes += [(32, 16, 2), (48, 12, 1), (64, 20, 1)]
    else:
        shapes += [(28, 20, 1)]
    for E, K, S in shapes:
        rc.set_option("embed.S", S)
        rc.set_option("embed.E", E)
        rc.set_option("embed.K", K)
        say(f"shape {variant} E={E} K={K} S={S}")
        outs.append(run_gpu(rc, *case, nsteps)[:2])
    for lo, hi in outs[1:]:
        assert np.array_equal(lo, outs[0][0]) and np.array_equal(hi, outs[0][1])


def test_resume_is_bitwise(rc):
    """embed(N1) then embed(N2) from its box equals embed(N1 + N2)."""
    kind, prm, lo, hi, pl, ph, dt = make_case("rd", 50000, np.float64, seed=9)
    say("resume")
    a_lo, a_hi, _ = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, 30)
    b_lo, b_hi, _ = run_gpu(rc, kind, prm, a_lo, a_hi, pl, ph, dt, 25, t0=30 * dt)
    c_lo, c_hi, _ = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, 55)
    assert np.array_equal(b_lo, c_lo) and np.array_equal(b_hi, c_hi)


def test_repeat_is_bitwise(rc):
    kind, prm, lo, hi, pl, ph, dt = make_case("ctm", 70001, np.float32, seed=10)
    say("repeat")
    a = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, 33)
    b = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, 33)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("S", [1, 2])
@pytest.mark.parametrize("nsteps", [8, 16, 17, 40])
def test_in_place_output(rc, nsteps, S):
    """r may alias x, whatever the number of passes."""
    kind, prm, lo, hi, pl, ph, dt = make_case("ctm", 9000, np.float64, seed=11)
    rc.set_option("embed.S", S)
    rc.set_option("embed.E", 4)
    rc.set_option("embed.K", 8)
    ref = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, nsteps)
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    say(f"in place N={nsteps}")
    rc.embed(kind, prm, x_lo, x_hi, dt, nsteps, r_lo=x_lo, r_hi=x_hi)
    assert rc.sync() == R.REACH_OK
    assert np.array_equal(to_host(x_lo), ref[0]) and np.array_equal(to_host(x_hi), ref[1])


def test_zero_steps_copies_box(rc):
    kind, prm, lo, hi, pl, ph, dt = make_case("rd", 777, np.float64, seed=12)
    g_lo, g_hi, st = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, 0)
    assert st == R.REACH_OK and np.array_equal(g_lo, lo) and np.array_equal(g_hi, hi)


@pytest.mark.parametrize("S", [1, 2])
def test_nonfinite_and_order_reported(rc, S):
    kind, prm, lo, hi, pl, ph, dt = make_case("rd", 100000, np.float64, seed=13)
    rc.set_option("embed.S", S)
    bad = lo.copy()
    bad[50000] = np.nan
    say("nan input")
    _, _, st = run_gpu(rc, kind, prm, bad, hi, pl, ph, dt, 5)
    assert st == R.REACH_E_NONFINITE
    say("lower above upper")
    _, _, st = run_gpu(rc, kind, prm, hi + 1.0, lo, pl, ph, dt, 5)
    assert st == R.REACH_E_ORDER
    _, _, st = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, 5)
    assert st == R.REACH_OK


@pytest.mark.parametrize("n", [1, 64, 700, 2048])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_single_window_flags_from_the_paired_waves(rc, n, dtype):
    """A chain one window holds runs as one block of two waves (lower, upper)
    that compare their boxes themselves: order and non-finite flags still
    reach the status word, and a clean box matches the oracle."""
    kind, prm, lo, hi, pl, ph, dt = make_case("ctm", n, dtype, seed=n + 17)
    dcode = R.REACH_F64 if dtype == np.float64 else R.REACH_F32
    plan = R.reach_plan_embed(rc.ctx, R.make_system(kind, n, prm, 0), dcode, 7)
    assert plan["S"] == 1 and plan["passes"] == 1 and plan["halo"] == 0
    say(f"paired single window n={n}")
    g_lo, g_hi, st = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, 7)
    assert st == R.REACH_OK
    o_lo, o_hi = oracle.embed_rk4(kind, prm, lo.astype(np.float64), hi.astype(np.float64), dt=dt,
                                  nsteps=7)
    assert_rel(g_lo, o_lo, RTOL[np.dtype(dtype)], "lower")
    assert_rel(g_hi, o_hi, RTOL[np.dtype(dtype)], "upper")
    crossed_lo, crossed_hi = lo.copy(), hi.copy()
    crossed_lo[n // 2], crossed_hi[n // 2] = hi[n // 2] + 5, lo[n // 2]
    _, _, st = run_gpu(rc, kind, prm, crossed_lo, crossed_hi, pl, ph, dt, 7)
    assert st == R.REACH_E_ORDER
    bad = lo.copy()
    bad[n - 1] = np.inf
    _, _, st = run_gpu(rc, kind, prm, bad, hi, pl, ph, dt, 7)
    assert st == R.REACH_E_NONFINITE
    assert rc.sync() == R.REACH_OK


def test_invalid_arguments_rejected(rc):
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    sys_ok = R.make_system(R.REACH_RD, 16, (1.0,), 1)
    p = torch.zeros(1, dtype=torch.float64, device="cuda")

    def call(sys, dt=0.1, nsteps=1, pl=p, ph=p, dtype=R.REACH_F64):
        return R.lib().reach_embed_rk4(rc.ctx, R.ctypes.byref(sys), dtype, x.data_ptr(),
                                       x.data_ptr(), R._ptr(pl), R._ptr(ph), 0.0, dt, nsteps,
                                       x.data_ptr(), x.data_ptr(), None, 0, None)
    assert call(sys_ok) == R.REACH_OK
    assert call(sys_ok, dt=0.0) == R.REACH_E_INVAL
    assert call(sys_ok, dt=float("nan")) == R.REACH_E_INVAL
    assert call(sys_ok, nsteps=-1) == R.REACH_E_INVAL
    assert call(sys_ok, pl=None) == R.REACH_E_INVAL
    assert call(sys_ok, dtype=7) == R.REACH_E_INVAL
    assert call(R.make_system(R.REACH_RD, 0, (1.0,), 1)) == R.REACH_E_INVAL
    assert call(R.make_system(R.REACH_RD, 16, (1.0,), 3)) == R.REACH_E_INVAL
    assert call(R.make_system(9, 16, (1.0,), 1)) == R.REACH_E_INVAL
    assert call(R.make_system(R.REACH_RD, 16, (0.0,), 1)) == R.REACH_E_INVAL
    assert call(R.make_system(R.REACH_CTM, 16, workloads.CTM_PRM, 1)) == R.REACH_E_UNSUPPORTED
    big = R.make_system(R.REACH_CTM, 1 << 20, workloads.CTM_PRM, 0)
    y = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    st = R.lib().reach_embed_rk4(rc.ctx, R.ctypes.byref(big), R.REACH_F64, y.data_ptr(),
                                 y.data_ptr(), None, None, 0.0, 0.01, 100, y.data_ptr(),
                                 y.data_ptr(), None, 0, None)
    assert st == R.REACH_E_INVAL          # multi-pass without workspace
    assert rc.sync() == R.REACH_OK


# --------------------------------------------------------- full-size configs

def test_ctm64_f64_embedding(rc):
    p = workloads.ctm64_f64()
    lo, hi = p.box()
    say("ctm64 embedding")
    g_lo, g_hi, st = run_gpu(rc, p.kind, p.prm, lo, hi, None, None, p.dt, p.nsteps)
    assert st == R.REACH_OK
    o_lo, o_hi = oracle.embed_rk4(p.kind, p.prm, lo, hi, dt=p.dt, nsteps=p.nsteps)
    assert_rel(g_lo, o_lo, 1e-12, "lower")
    assert_rel(g_hi, o_hi, 1e-12, "upper")


def _window_check(g_lo, g_hi, p, windows, rtol, pl=None, ph=None):
    for a, b in windows:
        o_lo, o_hi = oracle.embed_window(p.kind, p.prm, lambda i0, c: p.box(i0, c), p.n, a, b,
                                         p.nsteps, pl, ph, dt=p.dt)
        assert_rel(g_lo[a:b], o_lo, rtol, f"lower [{a},{b})")
        assert_rel(g_hi[a:b], o_hi, rtol, f"upper [{a},{b})")


def _windows(n, count, width, seed):
    rng = np.random.default_rng(seed)
    starts = rng.integers(0, n - width, count)
    return [(0, width), (n - width, n)] + [(int(s), int(s) + width) for s in starts]


def test_rd_2p26_f64_light_cone_windows(rc):
    """RD, n = 2^26, FP64, 1000 steps: the benchmark launch; sampled windows
    against the oracle's light-cone windows (bitwise equal to a whole-chain run)."""
    p = workloads.rd_2p26_f64()
    say("rd 2^26 inputs")
    lo, hi = p.box()
    pl, ph = p.inputs()
    say("rd 2^26 GPU run")
    g_lo, g_hi, st = run_gpu(rc, p.kind, p.prm, lo, hi, pl, ph, p.dt, p.nsteps)
    assert st == R.REACH_OK
    del lo, hi
    say("rd 2^26 oracle windows")
    _window_check(g_lo, g_hi, p, _windows(p.n, 64, 4096, 1), 1e-12, pl, ph)


def test_ctm_2p31_f32_light_cone_windows(rc):
    """CTM, n = 2^31 (64-bit indexing), FP32, 200 steps, windows vs oracle."""
    p = workloads.ctm_2p31_f32()
    free, _ = torch.cuda.mem_get_info()
    need = 6 * p.n * 4 + (1 << 30)
    if free < need:
        pytest.skip(f"needs {need >> 30} GiB of free device memory")
    say("ctm 2^31 inputs")
    lo = np.empty(p.n, dtype=np.float32)
    hi = np.empty(p.n, dtype=np.float32)
    p.box(out=(lo, hi))
    x_lo, x_hi = torch.from_numpy(lo).to("cuda"), torch.from_numpy(hi).to("cuda")
    del lo, hi
    say("ctm 2^31 GPU run")
    r_lo, r_hi = rc.embed(p.kind, p.prm, x_lo, x_hi, p.dt, p.nsteps, r_lo=x_lo, r_hi=x_hi)
    assert rc.sync() == R.REACH_OK
    say("ctm 2^31 oracle windows")
    wins = _windows(p.n, 64, 4096, 2)
    # the last cells sit past 2^31 - 1: exercise 64-bit indexing explicitly
    wins.append((p.n - 4096, p.n - 3840))
    for a, b in wins:
        g_lo = r_lo[a:b].cpu().numpy()
        g_hi = r_hi[a:b].cpu().numpy()
        o_lo, o_hi = oracle.embed_window(p.kind, p.prm, lambda i0, c: p.box(i0, c), p.n, a, b,
                                         p.nsteps, dt=p.dt)
        assert_rel(g_lo, o_lo, 1e-5, f"lower [{a},{b})")
        assert_rel(g_hi, o_hi, 1e-5, f"upper [{a},{b})")
    del x_lo, x_hi, r_lo, r_hi
    rc._ws = None
    torch.cuda.empty_cache()


def test_autotuner_picks_a_built_shape_and_keeps_results(rc):
    """The autotuner's choice changes speed only: results stay bitwise equal."""
    kind, prm, lo, hi, pl, ph, dt = make_case("rd", 300001, np.float64, seed=21)
    x_lo, x_hi, p_lo, p_hi = to_dev(lo), to_dev(hi), to_dev(pl), to_dev(ph)
    ref = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, 40)
    sysd = R.make_system(kind, lo.size, prm, 1)
    ws = torch.empty(2 * lo.size * 8, dtype=torch.uint8, device="cuda")
    r_lo, r_hi = torch.empty_like(x_lo), torch.empty_like(x_hi)
    say("autotune")
    best = R.reach_autotune_embed(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, p_lo, p_hi, dt, 16,
                                  r_lo, r_hi, ws, ws.numel())
    assert best["E"] in (4, 8, 12, 16, 24, 28, 32) and 8 * best["K"] < 64 * best["E"]
    assert best["S"] in (1, 2) and best["fs_per_state_step"] > 0
    plan = R.reach_plan_embed(rc.ctx, sysd, R.REACH_F64, 40)
    # the plan keeps the tuned pass count and spreads the 40 steps evenly
    passes = -(-40 // best["K"])
    assert (plan["E"], plan["K"], plan["S"]) == (best["E"], -(-40 // passes), best["S"])
    assert plan["passes"] == passes
    got = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, 40)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("variant,n", [("ctm", 7), ("rd", 40000), ("lin3", 3000)])
def test_reach_tube_slots_equal_single_runs(rc, variant, n):
    """Slot k of the tube is the box after (k+1)*every steps, bitwise."""
    kind, prm, lo, hi, pl, ph, dt = make_case(variant, n, np.float64, seed=31)
    every, slots = 9, 5
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    dev = lambda a: None if a is None else to_dev(a)
    sysd = R.make_system(kind, n, prm, 0 if pl is None else pl.size)
    tube_lo = torch.empty(slots * n, dtype=torch.float64, device="cuda")
    tube_hi = torch.empty_like(tube_lo)
    ws = torch.empty(2 * n * 8, dtype=torch.uint8, device="cuda")
    say(f"tube {variant} n={n}")
    R.reach_embed_rk4_tube(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, dev(pl), dev(ph), 0.0, dt,
                           every * slots, every, tube_lo, tube_hi, ws, ws.numel())
    assert rc.sync() == R.REACH_OK
    t_lo, t_hi = to_host(tube_lo).reshape(slots, n), to_host(tube_hi).reshape(slots, n)
    for k in range(slots):
        g = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, (k + 1) * every)
        assert np.array_equal(t_lo[k], g[0]) and np.array_equal(t_hi[k], g[1])
    o_lo, o_hi = run_oracle(kind, prm, lo, hi, pl, ph, dt, 2 * every)
    assert_rel(t_lo[1], o_lo, 1e-12, "slot 1 lower")
    assert_rel(t_hi[1], o_hi, 1e-12, "slot 1 upper")


def test_horizon_t1_equals_step_count(rc):
    """embed(..., t1=...) takes round((t1 - t0) / dt) steps."""
    kind, prm, lo, hi, pl, ph, dt = make_case("rd", 3000, np.float64, seed=44)
    say("horizon t1")
    a = rc.embed(kind, prm, to_dev(lo), to_dev(hi), dt, 30, p_lo=to_dev(pl), p_hi=to_dev(ph))
    b = rc.embed(kind, prm, to_dev(lo), to_dev(hi), dt, p_lo=to_dev(pl), p_hi=to_dev(ph),
                 t0=1.0, t1=1.0 + 30 * dt)
    assert rc.sync() == R.REACH_OK
    assert np.array_equal(to_host(a[0]), to_host(b[0])) and np.array_equal(to_host(a[1]), to_host(b[1]))
    with pytest.raises(ValueError):
        rc.embed(kind, prm, to_dev(lo), to_dev(hi), dt, p_lo=to_dev(pl), p_hi=to_dev(ph),
                 t0=0.0, t1=0.123 * dt + dt)


def test_reach_log_writes_one_json_record_per_call(capfd, monkeypatch):
    """REACH_LOG: a context created with it set writes the call and its launch
    plan as one JSON line on stderr per call."""
    import json
    monkeypatch.setenv("REACH_LOG", "1")
    r = R.Reach(0)
    try:
        kind, prm, lo, hi, pl, ph, dt = make_case("rd", 5000, np.float64, seed=31)
        say("REACH_LOG embed + montecarlo")
        capfd.readouterr()
        r.embed(kind, prm, to_dev(lo), to_dev(hi), dt, 30, p_lo=to_dev(pl), p_hi=to_dev(ph))
        r.montecarlo(kind, prm, to_dev(lo[:300]), to_dev(hi[:300]), dt, 5, 40, 3,
                     p_lo=to_dev(pl[:300]), p_hi=to_dev(ph[:300]))
        assert r.sync() == R.REACH_OK
        err = capfd.readouterr().err
        plan = R.reach_plan_embed(r.ctx, R.make_system(kind, 5000, prm, pl.size), R.REACH_F64, 30)
    finally:
        r.close()
    recs = [json.loads(l[len("reach: "):]) for l in err.splitlines() if l.startswith("reach: {")]
    assert [x["call"] for x in recs] == ["embed", "montecarlo"]
    e, m = recs
    assert (e["n"], e["nsteps"], e["dtype"], e["kind"]) == (5000, 30, "f64", kind)
    assert (e["E"], e["K"], e["S"], e["passes"]) == (plan["E"], plan["K"], plan["S"], plan["passes"])
    assert (m["n"], m["m"], m["nsteps"]) == (300, 40, 5) and m["waves"] == 40


def test_default_plan_spreads_steps_evenly_over_its_passes(rc):
    """Without a forced K the plan keeps the default pass count and evens out
    the steps per pass (a smaller halo); results do not depend on it."""
    kind, prm, lo, hi, pl, ph, dt = make_case("rd", 200003, np.float64, seed=23)
    sysd = R.make_system(kind, lo.size, prm, 1)
    k_default = R.reach_plan_embed(rc.ctx, sysd, R.REACH_F64, 100000)["K"]
    for nsteps in (1, 7, k_default + 1, 3 * k_default - 1, 100):
        plan = R.reach_plan_embed(rc.ctx, sysd, R.REACH_F64, nsteps)
        passes = -(-nsteps // k_default)
        assert plan["passes"] == passes and plan["K"] == -(-nsteps // passes), (nsteps, plan)
    say("even passes vs forced K")
    a = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, k_default + 1)
    rc.set_option("embed.K", k_default)
    b = run_gpu(rc, kind, prm, lo, hi, pl, ph, dt, k_default + 1)
    rc.set_option("embed.K", 0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_autotune_cache_keys_the_input_mode_and_ignores_old_lines(tmp_path, monkeypatch):
    """REACH_AUTOTUNE_CACHE: entries carry the input mode (shared or per-cell
    inputs), so a shape tuned for one never reaches the other; lines of the
    older format without it are ignored; batch pack-width lines apply to
    their (kind, size) bucket."""
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    n = 300000
    b = n.bit_length() - 1
    cache = tmp_path / "tune.txt"
    cache.write_text(
        f"{arch} 2 0 {b} 4 3 2 1.0\n"                       # old format: ignored
        f"reach2 embed {arch} 2 0 {b} 0 16 6 1 1.0\n"       # RD FP64, shared input
        f"reach2 embed {arch} 2 0 {b} 1 8 5 1 1.0\n"        # RD FP64, per-cell inputs
        f"reach2 batch {arch} 1 4 2 1000\n")                # CTM, n in [16, 32): width 2
    monkeypatch.setenv("REACH_AUTOTUNE_CACHE", str(cache))
    r = R.Reach(0)
    try:
        shared = R.reach_plan_embed(r.ctx, R.make_system(R.REACH_RD, n, (1.0,), 1),
                                    R.REACH_F64, 60)
        cell = R.reach_plan_embed(r.ctx, R.make_system(R.REACH_RD, n, (1.0,), n),
                                  R.REACH_F64, 60)
        assert (shared["E"], shared["S"]) == (16, 1) and shared["passes"] == 10
        assert (cell["E"], cell["S"]) == (8, 1) and cell["passes"] == 12
        r.set_option("batch.pack", 1)
        p = workloads.small_problem(workloads.KIND_CTM, 20, 3, 30)
        qs = [R.make_query(p.kind, 20, p.prm, R.REACH_F64, 1 << 20, 1 << 20, 1 << 20, 1 << 20,
                           p.dt, 30) for _ in range(40)]
        plan = R.reach_plan_batch(r.ctx, qs, with_E=True)
        assert plan and all(E == 2 for E, _ in plan)
    finally:
        r.close()
