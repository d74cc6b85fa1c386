"""GPU parity of reach_montecarlo against the FP64 oracle (Monte Carlo method,
Sec. 2.1 / Algorithm 4) and its containment in the embedding box."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import RTOL, assert_rel, say, to_dev, to_host
from tests.test_gpu_embed import KIND, make_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2001_10635_amd")


@pytest.fixture(scope="module")
def rc():
    r = R.Reach(0)
    yield r
    r.close()


def run_mc(rc, kind, prm, lo, hi, pl, ph, dt, nsteps, m, seed, s0=0):
    dev = lambda a: None if a is None else to_dev(a)
    r_min, r_max = rc.montecarlo(kind, prm, dev(lo), dev(hi), dt, nsteps, m, seed, p_lo=dev(pl),
                                 p_hi=dev(ph), s0=s0)
    st = rc.sync()
    return to_host(r_min), to_host(r_max), st


def oracle_mc(kind, prm, lo, hi, pl, ph, dt, nsteps, m, seed, dtype, s0=0):
    f = lambda a: None if a is None else np.asarray(a, dtype=np.float64)
    return oracle.montecarlo(kind, prm, f(lo), f(hi), f(pl), f(ph), dt=dt, nsteps=nsteps, m=m,
                             seed=seed, s0=s0, ubits=53 if dtype == np.float64 else 24)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("variant", ["ctm", "rd", "rd_cell", "lin3", "lin3_cell"])
@pytest.mark.parametrize("n", [1, 3, 64, 100, 257, 1000, 1500, 2048])
def test_mc_matches_oracle(rc, variant, n, dtype):
    case = make_case(variant, n, dtype, seed=2000 + n)
    m, nsteps, seed = 48, 23, 31 + n
    say(f"mc {variant} n={n} {np.dtype(dtype).name}")
    g_min, g_max, st = run_mc(rc, *case, nsteps, m, seed)
    assert st == R.REACH_OK
    o_min, o_max = oracle_mc(*case, nsteps, m, seed, dtype)
    rt = RTOL[np.dtype(dtype)]
    assert_rel(g_min, o_min, rt, "min")
    assert_rel(g_max, o_max, rt, "max")


@pytest.mark.parametrize("variant", ["ctm", "rd", "rd_cell", "lin3", "lin3_cell"])
@pytest.mark.parametrize("n", [2100, 3000, 4000])
def test_mc_f32_wide_padded_matches_oracle(rc, variant, n):
    """FP32 chains of 2049-4095 cells: 64 cells per lane with the chain ending
    inside the wave (the per-cell boundary select of the widest lanes)."""
    case = make_case(variant, n, np.float32, seed=2000 + n)
    m, nsteps, seed = 32, 17, 31 + n
    say(f"mc {variant} n={n} float32")
    g_min, g_max, st = run_mc(rc, *case, nsteps, m, seed)
    assert st == R.REACH_OK
    o_min, o_max = oracle_mc(*case, nsteps, m, seed, np.float32)
    assert_rel(g_min, o_min, 1e-5, "min")
    assert_rel(g_max, o_max, 1e-5, "max")


def test_mc_f32_full_width_n4096(rc):
    case = make_case("ctm", 4096, np.float32, seed=3)
    say("mc ctm n=4096 f32")
    g_min, g_max, st = run_mc(rc, *case, 40, 32, 5)
    assert st == R.REACH_OK
    o_min, o_max = oracle_mc(*case, 40, 32, 5, np.float32)
    assert_rel(g_min, o_min, 1e-5, "min")
    assert_rel(g_max, o_max, 1e-5, "max")


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_mc_zero_steps_gives_raw_draws_bitwise(rc, dtype):
    """On the box [0, 1] with no steps each sample is U(s, j) itself."""
    n, m, seed = 70, 9, 20010638
    lo, hi = np.zeros(n, dtype), np.ones(n, dtype)
    say("mc raw draws")
    g_min, g_max, st = run_mc(rc, R.REACH_CTM, workloads.CTM_PRM, lo, hi, None, None, 0.01, 0, m,
                              seed)
    bits = 53 if dtype == np.float64 else 24
    U = np.array([[oracle.uniform(seed, s, j, bits) for j in range(n)] for s in range(m)])
    assert np.array_equal(g_min.astype(np.float64), U.min(axis=0))
    assert np.array_equal(g_max.astype(np.float64), U.max(axis=0))


def test_mc_sample_ranges_compose_bitwise(rc):
    case = make_case("rd", 300, np.float64, seed=6)
    say("mc ranges")
    a = run_mc(rc, *case, 30, 100, 7, s0=0)
    b = run_mc(rc, *case, 30, 157, 7, s0=100)
    w = run_mc(rc, *case, 30, 257, 7, s0=0)
    assert np.array_equal(np.minimum(a[0], b[0]), w[0])
    assert np.array_equal(np.maximum(a[1], b[1]), w[1])
    assert np.all(w[0] <= a[0]) and np.all(w[1] >= a[1])


def test_mc_wave_count_invariance_bitwise(rc):
    case = make_case("ctm", 200, np.float32, seed=8)
    outs = []
    # 6, 7 and 65 leave 2, 3 and 1 waves in the last workgroup's fold
    for waves in (1, 6, 7, 64, 65, 0):
        rc.set_option("mc.waves", waves)
        say(f"mc waves={waves}")
        outs.append(run_mc(rc, *case, 25, 300, 9)[:2])
    rc.set_option("mc.waves", 0)
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_mc_two_pass_reduction_at_the_wave_cap_bitwise(rc):
    """4096 waves (1024 workgroup partials: 4 chunks of 256, reduced in two
    passes) and 100 waves (25 partials, one pass) give the same box; a wave
    count above the cap is clamped."""
    case = make_case("rd", 130, np.float64, seed=12)
    outs = []
    for waves in (100, 4096, 10000):
        rc.set_option("mc.waves", waves)
        say(f"mc waves={waves} m=5000")
        outs.append(run_mc(rc, *case, 10, 5000, 13)[:2])
    rc.set_option("mc.waves", 0)
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_mc_rejects_bad_requests(rc):
    x = torch.zeros(5000, dtype=torch.float32, device="cuda")
    s = R.make_system(R.REACH_CTM, 5000, workloads.CTM_PRM, 0)
    with pytest.raises(R.ReachError) as e:
        R.reach_workspace_bytes(rc.ctx, s, R.REACH_F32, 10)
    st = R.lib().reach_montecarlo(rc.ctx, R.ctypes.byref(s), R.REACH_F32, x.data_ptr(),
                                  x.data_ptr(), None, None, 0.0, 0.01, 5, 10, 1, x.data_ptr(),
                                  x.data_ptr(), x.data_ptr(), 1 << 20, None)
    assert st == R.REACH_E_UNSUPPORTED
    s2 = R.make_system(R.REACH_CTM, 100, workloads.CTM_PRM, 0)
    st = R.lib().reach_montecarlo(rc.ctx, R.ctypes.byref(s2), R.REACH_F32, x.data_ptr(),
                                  x.data_ptr(), None, None, 0.0, 0.01, 5, 0, 1, x.data_ptr(),
                                  x.data_ptr(), x.data_ptr(), 1 << 20, None)
    assert st == R.REACH_E_INVAL
    assert rc.sync() == R.REACH_OK


def test_ctm64_f64_mc_1000_samples(rc):
    p = workloads.ctm64_f64()
    lo, hi = p.box()
    say("ctm64 MC")
    g_min, g_max, st = run_mc(rc, p.kind, p.prm, lo, hi, None, None, p.dt, p.nsteps, p.m, p.seed)
    assert st == R.REACH_OK
    o_min, o_max = oracle.montecarlo(p.kind, p.prm, lo, hi, dt=p.dt, nsteps=p.nsteps, m=p.m,
                                     seed=p.seed)
    assert_rel(g_min, o_min, 1e-12, "min")
    assert_rel(g_max, o_max, 1e-12, "max")
    e_lo, e_hi = oracle.embed_rk4(p.kind, p.prm, lo, hi, dt=p.dt, nsteps=p.nsteps)
    assert np.all(g_min >= e_lo) and np.all(g_max <= e_hi)


def test_mc_ctm4096_f32(rc):
    """n = 4096 FP32, 500 steps.  Oracle parity on a 4096-sample prefix at the
    default wave count: 8 waves per CU (2048 on 256 CUs), so every wave
    integrates two samples (its second folds into the partials it wrote for the
    first) and the workgroup partials span two chunks of the reduction, which
    then takes its second pass.  Then the full 2^20 samples with containment in
    the FP64 embedding box, within the parity slack and counted without it."""
    p = workloads.mc_ctm4096_f32()
    lo, hi = p.box()
    m_sub = 4096
    rc.set_option("mc.waves", 0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    waves = min(8 * cus, 4096, m_sub)
    assert m_sub > waves, "prefix must give some wave a second sample"
    assert -(-waves // 4) > 256, "workgroup partials must span more than one reduction chunk"
    say(f"mc ctm4096 MC prefix m={m_sub} waves={waves}")
    g_min, g_max, st = run_mc(rc, p.kind, p.prm, lo, hi, None, None, p.dt, p.nsteps, m_sub, p.seed)
    assert st == R.REACH_OK
    o_min, o_max = oracle.montecarlo(p.kind, p.prm, lo.astype(np.float64), hi.astype(np.float64),
                                     dt=p.dt, nsteps=p.nsteps, m=m_sub, seed=p.seed, ubits=24)
    e1 = assert_rel(g_min, o_min, 1e-5, "min")
    e2 = assert_rel(g_max, o_max, 1e-5, "max")
    say(f"mc ctm4096 prefix max rel err min {e1:.2e} max {e2:.2e}")
    say("mc ctm4096 MC full")
    f_min, f_max, st = run_mc(rc, p.kind, p.prm, lo, hi, None, None, p.dt, p.nsteps, p.m, p.seed)
    assert st == R.REACH_OK
    assert np.all(f_min <= g_min) and np.all(f_max >= g_max)    # prefix nesting
    say("mc ctm4096 FP64 embedding box")
    e_lo, e_hi, st = run_embed64(rc, p, lo, hi)
    assert st == R.REACH_OK
    o_elo, o_ehi = oracle.embed_rk4(p.kind, p.prm, lo.astype(np.float64), hi.astype(np.float64),
                                    dt=p.dt, nsteps=p.nsteps)
    assert_rel(e_lo, o_elo, 1e-12, "embedding lower")
    assert_rel(e_hi, o_ehi, 1e-12, "embedding upper")
    slack = 1e-5 * np.maximum(np.abs(e_lo), 1.0)
    assert np.all(f_min >= e_lo - slack) and np.all(f_max <= e_hi + slack)
    exact = int(np.count_nonzero((f_min < e_lo) | (f_max > e_hi)))
    # the oracle's own samples (FP64 arithmetic) lie inside the oracle box exactly
    assert np.all(o_min >= o_elo) and np.all(o_max <= o_ehi)
    say(f"mc ctm4096 containment: {exact} of {p.n} cells outside without slack")


def run_embed64(rc, p, lo, hi):
    r_lo, r_hi = rc.embed(p.kind, p.prm, to_dev(lo.astype(np.float64)),
                          to_dev(hi.astype(np.float64)), p.dt, p.nsteps)
    return to_host(r_lo), to_host(r_hi), rc.sync()
