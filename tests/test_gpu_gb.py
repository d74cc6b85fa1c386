"""GPU parity of reach_growth_bound against the FP64 oracle (contraction /
growth-bound method, Sec. 2.1 / Algorithm 2)."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import RTOL, assert_rel, say, to_dev, to_host
from tests.test_gpu_embed import make_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2001_10635_amd")


@pytest.fixture(scope="module")
def rc():
    r = R.Reach(0)
    yield r
    r.close()


@pytest.fixture(autouse=True)
def _reset(rc):
    rc.set_option("gb.E", 0)
    rc.set_option("gb.K", 0)
    yield
    rc.set_option("gb.E", 0)
    rc.set_option("gb.K", 0)


def run_gb(rc, kind, prm, lo, hi, pl, ph, dt, nsteps):
    dev = lambda a: None if a is None else to_dev(a)
    r_lo, r_hi = rc.growth_bound(kind, prm, dev(lo), dev(hi), dt, nsteps, p_lo=dev(pl),
                                 p_hi=dev(ph))
    return to_host(r_lo), to_host(r_hi), rc.sync()


def oracle_gb(kind, prm, lo, hi, pl, ph, dt, nsteps):
    f = lambda a: None if a is None else np.asarray(a, dtype=np.float64)
    return oracle.growth_bound(kind, prm, f(lo), f(hi), f(pl), f(ph), dt=dt, nsteps=nsteps)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("variant", ["ctm", "rd", "rd_cell", "lin3", "lin3_cell"])
@pytest.mark.parametrize("n", [1, 5, 64, 65, 1000, 2049, 5000])
def test_gb_matches_oracle(rc, variant, n, dtype):
    case = make_case(variant, n, dtype, seed=3000 + n)
    say(f"gb {variant} n={n} {np.dtype(dtype).name}")
    g_lo, g_hi, st = run_gb(rc, *case, 33)
    assert st == R.REACH_OK
    o_lo, o_hi = oracle_gb(*case, 33)
    rt = RTOL[np.dtype(dtype)]
    assert_rel(g_lo, o_lo, rt, "lower")
    assert_rel(g_hi, o_hi, rt, "upper")


@pytest.mark.parametrize("E,K", [(1, 1), (4, 5), (8, 8), (16, 12), (24, 20), (28, 13), (32, 9)])
@pytest.mark.parametrize("variant", ["ctm", "rd", "lin3_cell"])
def test_gb_multitile_matches_oracle(rc, variant, E, K):
    n, nsteps = 4001, 47
    case = make_case(variant, n, np.float64, seed=88)
    rc.set_option("gb.E", E)
    rc.set_option("gb.K", K)
    say(f"gb multitile {variant} E={E} K={K}")
    g_lo, g_hi, st = run_gb(rc, *case, nsteps)
    assert st == R.REACH_OK
    o_lo, o_hi = oracle_gb(*case, nsteps)
    assert_rel(g_lo, o_lo, 1e-12, "lower")
    assert_rel(g_hi, o_hi, 1e-12, "upper")


def test_gb_contains_embedding_box(rc):
    kind, prm, lo, hi, pl, ph, dt = make_case("rd", 30000, np.float64, seed=89)
    g_lo, g_hi, _ = run_gb(rc, kind, prm, lo, hi, pl, ph, dt, 60)
    e_lo, e_hi = rc.embed(kind, prm, to_dev(lo), to_dev(hi), dt, 60, p_lo=to_dev(pl),
                          p_hi=to_dev(ph))
    assert rc.sync() == R.REACH_OK
    assert np.all(g_lo <= to_host(e_lo) + 1e-12) and np.all(g_hi >= to_host(e_hi) - 1e-12)


def test_gb_rd_2p26_f64_light_cone_windows(rc):
    """Growth bound on the 2^26-cell RD chain, 1000 steps, sampled windows."""
    p = workloads.rd_2p26_f64()
    lo, hi = p.box()
    pl, ph = p.inputs()
    say("gb rd 2^26 GPU run")
    g_lo, g_hi, st = run_gb(rc, p.kind, p.prm, lo, hi, pl, ph, p.dt, p.nsteps)
    assert st == R.REACH_OK
    rng = np.random.default_rng(3)
    r = 4 * p.nsteps
    for a in [0, p.n - 256] + [int(v) for v in rng.integers(0, p.n - 256, 4)]:
        b = a + 256
        i0, i1 = max(0, a - r), min(p.n, b + r)
        w_lo, w_hi = p.box(i0, i1 - i0)
        o_lo, o_hi = oracle.growth_bound(p.kind, p.prm, w_lo, w_hi, pl, ph, dt=p.dt,
                                         nsteps=p.nsteps, n_total=p.n, g0=i0)
        assert_rel(g_lo[a:b], o_lo[a - i0:b - i0], 1e-12, f"lower [{a},{b})")
        assert_rel(g_hi[a:b], o_hi[a - i0:b - i0], 1e-12, f"upper [{a},{b})")
