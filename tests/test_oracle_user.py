"""Pins of the oracle's user decomposition path (a chain system given as C
source text, Sec. 2.1: any decomposition function yields an embedding).
Restating a built-in system as user text must give the built-in oracle
result bitwise; the nonlinear sine chain is checked for the decomposition
function's defining properties and for soundness against sampled
trajectories."""
import numpy as np
import pytest

import oracle
import workloads
from tests import user_sources as us

CTM_PRM = workloads.CTM_PRM


@pytest.fixture(scope="module")
def users():
    return {k: oracle.UserSystem(getattr(us, k)) for k in ("LIN3", "CTM", "RD", "SINE")}


@pytest.mark.parametrize("coef", [(-0.5, -1.0, 0.75, -1.5), (0.3, -0.9, -0.2, 0.7)])
@pytest.mark.parametrize("inputs", ["none", "scalar", "cell"])
def test_user_lin3_equals_builtin_bitwise(users, coef, inputs):
    rng = np.random.default_rng(31)
    n = 57
    lo = rng.uniform(-1, 1, n)
    hi = lo + rng.uniform(0, 0.5, n)
    pl = ph = None
    if inputs == "scalar":
        pl, ph = np.array([-0.25]), np.array([0.5])
    elif inputs == "cell":
        pl = rng.uniform(-0.3, 0.0, n)
        ph = pl + rng.uniform(0.0, 0.6, n)
    u = oracle.embed_rk4_user(users["LIN3"], coef, lo, hi, pl, ph, dt=0.05, nsteps=40)
    b = oracle.embed_rk4(oracle.LIN3, coef, lo, hi, pl, ph, dt=0.05, nsteps=40)
    assert np.array_equal(u[0], b[0]) and np.array_equal(u[1], b[1])


def test_user_ctm_equals_builtin_bitwise_whole_and_window(users):
    p = workloads.small_problem(oracle.CTM, 300, 33, 30)
    lo, hi = p.box()
    u = oracle.embed_rk4_user(users["CTM"], CTM_PRM, lo, hi, dt=p.dt, nsteps=p.nsteps)
    b = oracle.embed_rk4(oracle.CTM, CTM_PRM, lo, hi, dt=p.dt, nsteps=p.nsteps)
    assert np.array_equal(u[0], b[0]) and np.array_equal(u[1], b[1])
    for g0, ln in ((0, 80), (100, 90), (220, 80)):      # windows touching each end
        u = oracle.embed_rk4_user(users["CTM"], CTM_PRM, lo[g0:g0 + ln], hi[g0:g0 + ln],
                                  dt=p.dt, nsteps=p.nsteps, n_total=p.n, g0=g0)
        b = oracle.embed_rk4(oracle.CTM, CTM_PRM, lo[g0:g0 + ln], hi[g0:g0 + ln], dt=p.dt,
                             nsteps=p.nsteps, n_total=p.n, g0=g0)
        assert np.array_equal(u[0], b[0]) and np.array_equal(u[1], b[1])


def test_user_rd_equals_builtin_bitwise(users):
    p = workloads.small_problem(oracle.RD, 200, 34, 50)
    lo, hi = p.box()
    pl, ph = p.inputs()
    u = oracle.embed_rk4_user(users["RD"], p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps)
    b = oracle.embed_rk4(oracle.RD, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps)
    assert np.array_equal(u[0], b[0]) and np.array_equal(u[1], b[1])


def _sine_case(n, seed):
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-3.0, 3.0, n)
    hi = lo + rng.uniform(0.0, 0.8, n)
    pl, ph = np.array([-0.2]), np.array([0.3])
    return lo, hi, pl, ph


def test_user_sine_degenerate_box_is_the_trajectory(users):
    lo, _, pl, _ = _sine_case(40, 35)
    r = oracle.embed_rk4_user(users["SINE"], us.SINE_PRM, lo, lo, pl, pl, dt=0.05, nsteps=60)
    t = oracle.f_rk4_user(users["SINE"], us.SINE_PRM, lo, pl, dt=0.05, nsteps=60)
    assert np.array_equal(r[0], r[1]) and np.array_equal(r[0], t)


def test_user_sine_trajectory_matches_a_reference_solver(users):
    """x' = -a x + b sin(x_{i-1}) + c u integrated by scipy's DOP853; RK4 with a
    small step agrees to its fourth-order error."""
    from scipy.integrate import solve_ivp
    a, b, c = us.SINE_PRM
    lo, _, _, _ = _sine_case(12, 36)
    u = 0.1

    def rhs(_, x):
        xm = np.concatenate([[0.0], x[:-1]])
        return -a * x + b * np.sin(xm) + c * u

    ref = solve_ivp(rhs, (0.0, 2.0), lo, method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    got = oracle.f_rk4_user(users["SINE"], us.SINE_PRM, lo, [u], dt=0.01, nsteps=200)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9)


def test_user_sine_box_contains_sampled_trajectories(users):
    n, dt, N = 30, 0.05, 60
    lo, hi, pl, ph = _sine_case(n, 37)
    r_lo, r_hi = oracle.embed_rk4_user(users["SINE"], us.SINE_PRM, lo, hi, pl, ph, dt=dt,
                                       nsteps=N)
    assert np.all(r_lo <= r_hi)
    rng = np.random.default_rng(38)
    for _ in range(64):
        x0 = lo + rng.uniform(0, 1, n) * (hi - lo)
        u = pl + rng.uniform() * (ph - pl)
        x = oracle.f_rk4_user(users["SINE"], us.SINE_PRM, x0, u, dt=dt, nsteps=N)
        assert np.all(x >= r_lo - 1e-12) and np.all(x <= r_hi + 1e-12)


def test_user_sine_box_is_tighter_than_trivially_wide(users):
    """The decomposition is not the trivial one: an initial box of width 0
    except one cell keeps far cells exact."""
    n = 20
    lo = np.linspace(-1, 1, n)
    hi = lo.copy()
    hi[10] += 0.5
    r_lo, r_hi = oracle.embed_rk4_user(users["SINE"], us.SINE_PRM, lo, hi, [0.0], [0.0],
                                       dt=0.05, nsteps=4)
    # cells below 10 never see the widened cell (coupling runs i-1 -> i only)
    assert np.array_equal(r_lo[:10], r_hi[:10])
    assert np.all(r_hi[10:] - r_lo[10:] > 0)


@pytest.mark.parametrize("name,kind", [("CTM", oracle.CTM), ("RD", oracle.RD)])
def test_user_montecarlo_equals_builtin_bitwise(users, name, kind):
    p = workloads.small_problem(kind, 40, 39, 25)
    lo, hi = p.box()
    pl, ph = p.inputs()
    u = oracle.montecarlo_user(users[name], p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps,
                               m=50, seed=9)
    b = oracle.montecarlo(kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps, m=50, seed=9)
    assert np.array_equal(u[0], b[0]) and np.array_equal(u[1], b[1])


def test_user_sine_montecarlo_samples_are_trajectories_inside_the_box(users):
    n, dt, N = 24, 0.05, 40
    lo, hi, pl, ph = _sine_case(n, 40)
    mn, mx, smp = oracle.montecarlo_user(users["SINE"], us.SINE_PRM, lo, hi, pl, ph, dt=dt,
                                         nsteps=N, m=64, seed=3, return_samples=True)
    assert np.array_equal(mn, smp.min(axis=0)) and np.array_equal(mx, smp.max(axis=0))
    e_lo, e_hi = oracle.embed_rk4_user(users["SINE"], us.SINE_PRM, lo, hi, pl, ph, dt=dt,
                                       nsteps=N)
    assert np.all(mn >= e_lo - 1e-12) and np.all(mx <= e_hi + 1e-12)
    for s in (0, 17, 63):     # each sample is the trajectory from its drawn point
        x0 = np.array([lo[j] + oracle.uniform(3, s, j) * (hi[j] - lo[j]) for j in range(n)])
        u = pl + oracle.uniform(3, s, n) * (ph - pl)
        t = oracle.f_rk4_user(users["SINE"], us.SINE_PRM, x0, u, dt=dt, nsteps=N)
        assert np.array_equal(t, smp[s])
