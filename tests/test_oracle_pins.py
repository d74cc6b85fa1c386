"""Pins of the FP64 oracle against facts outside its own code.

The paper prints no worked example (its result figures are not part of the
text and its tables hold only timings), so the oracle is pinned by
closed forms, exact rational arithmetic, invariants, convergence order,
library routines for the generic parts (Philox, min / max) and brute force on
tiny inputs.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import oracle
import workloads
from tests import closed_forms as cf

CTM_PRM = workloads.CTM_PRM


# ------------------------------------------------------------------ Philox

def _numpy_block(ctr, key):
    """Philox4x64-10 block at `ctr` from numpy's library generator.

    numpy advances its counter before producing a block, so start one below.
    """
    c = int(ctr[0]) | (int(ctr[1]) << 64) | (int(ctr[2]) << 128) | (int(ctr[3]) << 192)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=(c - 1) % (1 << 256))
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (12345, 0)),
    ((5, 7, 2, 0), (20010635, 0)),
    ((2**64 - 1, 3, 1, 9), (2**63 + 11, 77)),
    ((123456789, 2**40, 2, 0), (20010638, 0)),
])
def test_philox_matches_numpy(ctr, key):
    ref = _numpy_block(ctr, key)
    assert np.array_equal(oracle.philox(ctr, key), ref)
    assert np.array_equal(workloads.philox(ctr, key), ref)


def test_uniform_draw_layout():
    """U(s, j) = word j mod 4 of block (j // 4, s, 2, 0), top 53 or 24 bits."""
    seed = 20010638
    for s in (0, 1, 4097):
        for j in (0, 1, 2, 3, 4, 7, 4095, 4096):
            w = int(_numpy_block((j // 4, s, 2, 0), (seed, 0))[j % 4])
            assert oracle.uniform(seed, s, j, 53) == (w >> 11) * 2.0 ** -53
            assert oracle.uniform(seed, s, j, 24) == (w >> 40) * 2.0 ** -24


def test_workload_uniforms_match_numpy():
    seed = 77
    u = workloads.uniform(seed, 1, 5, 11)
    for k in range(11):
        i = 5 + k
        w = int(_numpy_block((i // 4, 0, 1, 0), (seed, 0))[i % 4])
        assert u[k] == (w >> 11) * 2.0 ** -53


# ------------------------------------------------------- linear closed forms

def _lin3_A(n, aL, aD, aR):
    return cf.tridiag(n, aL, aD, aR)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("coef", [(0.5, -1.25, 0.75, 2.0), (-0.375, -0.5, 1.5, -1.0)])
def test_lin3_trajectory_exact_rational(n, coef):
    """f-RK4 of a LIN3 chain equals R(hA)^N x0 + sum of R^k h S(hA) b u exactly."""
    aL, aD, aR, b = coef
    h, N, u = 0.125, 5, 0.5
    x0 = [0.75, -1.5, 2.25, 0.625][:n]
    A = _lin3_A(n, aL, aD, aR)
    exact = cf.to_float(cf.rk4_linear_exact(A, [b * u] * n, x0, h, N))
    got = oracle.f_rk4(oracle.LIN3, coef, x0, [u], dt=h, nsteps=N)
    np.testing.assert_allclose(got, exact, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_lin3_embedding_exact_rational(n):
    """Embedding of a mixed-sign LIN3 chain = the 2n linear system [[M, N], [N, M]]."""
    aL, aD, aR, b = -0.5, -1.0, 0.75, -1.5
    pl, ph = -0.25, 0.5
    h, N = 0.0625, 6
    lo = [0.5, -1.0, 0.25, 1.5][:n]
    hi = [0.75, -0.5, 1.25, 1.625][:n]
    big = cf.embedding_matrix(n, aL, aD, aR)
    bp, bn = (b if b > 0 else 0.0), (b if b < 0 else 0.0)
    # lower side input term: b+ p + b- ph ; upper side: b+ ph + b- p
    c = [Fraction(bp) * Fraction(pl) + Fraction(bn) * Fraction(ph)] * n + \
        [Fraction(bp) * Fraction(ph) + Fraction(bn) * Fraction(pl)] * n
    exact = cf.to_float(cf.rk4_linear_exact(big, c, lo + hi, h, N))
    r_lo, r_hi = oracle.embed_rk4(oracle.LIN3, (aL, aD, aR, b), lo, hi, [pl], [ph], dt=h,
                                  nsteps=N)
    np.testing.assert_allclose(np.concatenate([r_lo, r_hi]), exact, rtol=1e-14, atol=1e-14)


def test_lin3_per_cell_inputs_exact_rational():
    n, (aL, aD, aR, b) = 3, (0.25, -0.75, 0.5, 1.0)
    u = [0.5, -0.25, 0.125]
    h, N = 0.25, 4
    x0 = [1.0, 0.0, -1.0]
    exact = cf.to_float(cf.rk4_linear_exact(_lin3_A(n, aL, aD, aR), [b * v for v in u], x0,
                                            h, N))
    got = oracle.f_rk4(oracle.LIN3, (aL, aD, aR, b), x0, u, dt=h, nsteps=N)
    np.testing.assert_allclose(got, exact, rtol=1e-14, atol=1e-14)


def test_lin3_matches_matrix_exponential_to_fourth_order():
    """Error against expm(tA) x0 falls by ~2^4 per halving of the step."""
    n, coef = 6, (0.3, -1.1, 0.45, 0.0)
    A = np.diag([coef[1]] * n) + np.diag([coef[0]] * (n - 1), -1) + np.diag([coef[2]] * (n - 1), 1)
    x0 = np.linspace(-1.0, 1.0, n)
    T = 2.0
    ref = expm(T * A) @ x0
    errs = []
    for N in (10, 20, 40):
        got = oracle.f_rk4(oracle.LIN3, coef, x0, None, dt=T / N, nsteps=N)
        errs.append(np.max(np.abs(got - ref)))
    for e1, e2 in zip(errs, errs[1:]):
        assert 14.0 < e1 / e2 < 18.0


# ------------------------------------------------------------- RD pins

def test_rd_dirichlet_sine_mode_decays_by_stability_polynomial():
    """At amplitude 1e-8 the cubic term is below FP64 resolution, and the
    first Dirichlet mode of the diffusion stencil is an eigenvector with
    eigenvalue -4 sin^2(pi / (2 (n+1))) / h^2: x_N = R(lambda dt)^N x_0."""
    n, h, dt, N = 50, 1.0, 0.1, 100
    i = np.arange(n)
    x0 = 1e-8 * np.sin(np.pi * (i + 1) / (n + 1))
    lam = -4.0 * np.sin(np.pi / (2 * (n + 1))) ** 2 / h ** 2
    expect = cf.rk4_stability(lam * dt) ** N * x0
    got = oracle.f_rk4(oracle.RD, (h,), x0, [0.0], dt=dt, nsteps=N)
    np.testing.assert_allclose(got, expect, rtol=1e-12, atol=0)


def test_rd_spacing_scales_diffusion():
    n, h, dt, N = 20, 0.5, 0.01, 40
    i = np.arange(n)
    x0 = 1e-8 * np.sin(2 * np.pi * (i + 1) / (n + 1))   # second mode
    lam = -4.0 * np.sin(2 * np.pi / (2 * (n + 1))) ** 2 / h ** 2
    got = oracle.f_rk4(oracle.RD, (h,), x0, [0.0], dt=dt, nsteps=N)
    np.testing.assert_allclose(got, cf.rk4_stability(lam * dt) ** N * x0, rtol=1e-12)


def test_rd_single_cell_bernoulli_fourth_order():
    """n = 1, u = 0: x' = -2x - x^3 has a closed form; RK4 error ~ dt^4."""
    x0, T = 0.9, 2.0
    exact = cf.bernoulli_rd1(x0, T)
    errs = []
    for N in (20, 40, 80):
        got = oracle.f_rk4(oracle.RD, (1.0,), [x0], [0.0], dt=T / N, nsteps=N)[0]
        errs.append(abs(got - exact))
    assert errs[-1] < 1e-8
    for e1, e2 in zip(errs, errs[1:]):
        assert 14.0 < e1 / e2 < 18.0


def test_rd_input_enters_additively():
    x = np.array([0.3, -0.2, 0.7])
    f0 = oracle.rhs(oracle.RD, (1.0,), x, [0.0], use_f=True)
    f1 = oracle.rhs(oracle.RD, (1.0,), x, [0.1], use_f=True)
    np.testing.assert_allclose(f1 - f0, 0.1, rtol=0, atol=1e-15)
    # zero state, input u: f = u at every cell
    np.testing.assert_array_equal(oracle.rhs(oracle.RD, (1.0,), np.zeros(4), [0.25], use_f=True),
                                  0.25)


def test_rd_mirror_and_sign_symmetry():
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, 33)
    f = oracle.rhs(oracle.RD, (1.0,), x, [0.05], use_f=True)
    fr = oracle.rhs(oracle.RD, (1.0,), x[::-1], [0.05], use_f=True)
    np.testing.assert_allclose(fr[::-1], f, rtol=0, atol=1e-15)
    fn = oracle.rhs(oracle.RD, (1.0,), -x, [-0.05], use_f=True)
    np.testing.assert_array_equal(fn, -f)


def test_rd_chain_fourth_order_against_reference_solver():
    """n = 8 RD chain against a tight-tolerance DOP853 solution of the same ODE."""
    n, u, T = 8, 0.05, 1.0
    x0 = np.sin(np.pi * (np.arange(n) + 1) / (n + 1))

    def f(t, y):
        yp = np.concatenate([y[1:], [0.0]])
        ym = np.concatenate([[0.0], y[:-1]])
        return (ym - 2 * y + yp) - y ** 3 + u
    ref = solve_ivp(f, (0, T), x0, method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
    errs = []
    for N in (10, 20, 40):
        got = oracle.f_rk4(oracle.RD, (1.0,), x0, [u], dt=T / N, nsteps=N)
        errs.append(np.max(np.abs(got - ref)))
    for e1, e2 in zip(errs, errs[1:]):
        assert 13.0 < e1 / e2 < 19.0


# ------------------------------------------------------------- CTM pins

def _ctm_free_flow_A(n, v):
    """Free flow (v y_i below supply and capacity): F_i = v y_i, so
    f_i = v y_{i-1} - v y_i (no inflow into cell 0)."""
    A = cf.mat(n)
    for i in range(n):
        A[i][i] = Fraction(-v)
        if i > 0:
            A[i][i - 1] = Fraction(v)
    return A


def test_ctm_free_flow_regime_exact_rational():
    n, h, N = 4, 0.125, 6
    v, w, c, q = 0.5, 0.25, 40.0, 20.0
    x0 = [1.0, 0.5, 0.25, 0.75]
    exact = cf.to_float(cf.rk4_linear_exact(_ctm_free_flow_A(n, v), [0] * n, x0, h, N))
    got = oracle.f_rk4(oracle.CTM, (v, w, c, q), x0, None, dt=h, nsteps=N)
    np.testing.assert_allclose(got, exact, rtol=1e-14, atol=1e-15)


def test_ctm_congested_regime_exact_rational():
    """Near jam density the supply w (c - y_{i+1}) binds: F_i = w (c - y_{i+1})
    for i < n-1, and the free outflow v y_{n-1} sits below capacity."""
    n, h, N = 4, 0.0625, 4
    v, w, c, q = 0.5, 0.25, 40.0, 20.0
    x0 = [38.5, 39.0, 38.75, 39.5]
    A = cf.mat(n)
    b = [Fraction(0)] * n
    # f_0 = -w (c - y_1)
    A[0][1] = Fraction(w); b[0] = Fraction(-w * c)
    for i in range(1, n - 1):       # f_i = w (c - y_i) - w (c - y_{i+1})
        A[i][i] = Fraction(-w); A[i][i + 1] = Fraction(w)
    A[n - 1][n - 1] = Fraction(-w) - Fraction(v)   # f = w (c - y) - v y
    b[n - 1] = Fraction(w * c)
    exact = cf.to_float(cf.rk4_linear_exact(A, b, x0, h, N))
    got = oracle.f_rk4(oracle.CTM, (v, w, c, q), x0, None, dt=h, nsteps=N)
    np.testing.assert_allclose(got, exact, rtol=1e-14, atol=1e-13)


def test_ctm_capacity_regime():
    """All fluxes at capacity q: only cell 0 (no inflow) changes, at rate -q."""
    v, w, c, q = 1.0, 1.0, 100.0, 1.0
    x0 = np.array([15.0, 12.0, 18.0, 11.0, 16.0])
    got = oracle.f_rk4(oracle.CTM, (v, w, c, q), x0, None, dt=0.125, nsteps=8)
    expect = x0.copy()
    expect[0] -= q * 1.0
    np.testing.assert_array_equal(got, expect)


def test_ctm_mass_balance_and_zero_fixed_point():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 40, 100)
    f = oracle.rhs(oracle.CTM, CTM_PRM, x, use_f=True)
    v, w, c, q = CTM_PRM
    outflow = min(v * x[-1], q)
    assert abs(f.sum() + outflow) < 1e-11
    z = oracle.f_rk4(oracle.CTM, CTM_PRM, np.zeros(10), None, dt=0.01, nsteps=50)
    np.testing.assert_array_equal(z, 0.0)


def test_ctm_flux_uses_downstream_supply():
    """f_i depends on y_{i-1}, y_i, y_{i+1} exactly as the flux formula says."""
    v, w, c, q = CTM_PRM
    y = np.array([10.0, 30.0, 35.0, 5.0])
    F = [min(v * y[0], w * (c - y[1]), q), min(v * y[1], w * (c - y[2]), q),
         min(v * y[2], w * (c - y[3]), q), min(v * y[3], q)]
    expect = [0 - F[0], F[0] - F[1], F[1] - F[2], F[2] - F[3]]
    np.testing.assert_allclose(oracle.rhs(oracle.CTM, CTM_PRM, y, use_f=True), expect,
                               rtol=0, atol=1e-14)


# ------------------------------------------------------------- embedding

@pytest.mark.parametrize("kind", [oracle.CTM, oracle.RD])
def test_degenerate_box_collapses_to_trajectory(kind):
    p = workloads.small_problem(kind, 37, 5, 40)
    lo, _ = p.box()
    pl, ph = p.inputs()
    r_lo, r_hi = oracle.embed_rk4(kind, p.prm, lo, lo, pl, pl, dt=p.dt, nsteps=p.nsteps)
    assert np.array_equal(r_lo, r_hi)
    traj = oracle.f_rk4(kind, p.prm, lo, pl, dt=p.dt, nsteps=p.nsteps)
    assert np.array_equal(r_lo, traj)


@pytest.mark.parametrize("kind", [oracle.CTM, oracle.RD])
def test_cooperative_embedding_is_two_trajectories(kind):
    p = workloads.small_problem(kind, 29, 6, 60)
    lo, hi = p.box()
    pl, ph = p.inputs()
    r_lo, r_hi = oracle.embed_rk4(kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps)
    assert np.array_equal(r_lo, oracle.f_rk4(kind, p.prm, lo, pl, dt=p.dt, nsteps=p.nsteps))
    assert np.array_equal(r_hi, oracle.f_rk4(kind, p.prm, hi, ph, dt=p.dt, nsteps=p.nsteps))


@pytest.mark.parametrize("kind", [oracle.CTM, oracle.RD])
def test_lower_stays_below_upper_every_step(kind):
    p = workloads.small_problem(kind, 64, 7, 1)
    lo, hi = p.box()
    pl, ph = p.inputs()
    for _ in range(200):
        lo, hi = oracle.embed_rk4(kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=1)
        assert np.all(lo <= hi)


def test_lin3_decomposition_reduces_to_f_on_the_diagonal():
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, 17)
    coef = (-0.5, -1.0, 0.75, -1.5)
    d = oracle.rhs(oracle.LIN3, coef, x, [0.2], x, [0.2])
    f = oracle.rhs(oracle.LIN3, coef, x, [0.2], use_f=True)
    np.testing.assert_allclose(d, f, rtol=0, atol=1e-15)


def test_lin3_decomposition_monotonicity():
    """d is increasing in x off the diagonal and decreasing in xh."""
    rng = np.random.default_rng(4)
    coef = (-0.5, -1.0, 0.75, -1.5)
    x = rng.uniform(-1, 1, 9)
    xh = x + rng.uniform(0, 1, 9)
    base = oracle.rhs(oracle.LIN3, coef, x, [0.1], xh, [0.3])
    for j in range(9):
        e = np.zeros(9)
        e[j] = 0.01
        up = oracle.rhs(oracle.LIN3, coef, x + e, [0.1], xh, [0.3])
        mask = np.arange(9) != j
        assert np.all(up[mask] >= base[mask])
        dn = oracle.rhs(oracle.LIN3, coef, x, [0.1], xh + e, [0.3])
        assert np.all(dn <= base)


@pytest.mark.parametrize("kind", [oracle.CTM, oracle.RD])
def test_monte_carlo_samples_inside_embedding_box(kind):
    p = workloads.small_problem(kind, 48, 8, 100)
    lo, hi = p.box()
    pl, ph = p.inputs()
    r_lo, r_hi = oracle.embed_rk4(kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps)
    mn, mx, S = oracle.montecarlo(kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps, m=300,
                                  seed=9, return_samples=True)
    assert np.all(S >= r_lo) and np.all(S <= r_hi)
    assert np.all(mn >= r_lo) and np.all(mx <= r_hi)


def test_light_cone_window_is_bitwise_whole_chain():
    for kind in (oracle.CTM, oracle.RD):
        p = workloads.small_problem(kind, 700, 10, 25)
        lo, hi = p.box()
        pl, ph = p.inputs()
        r_lo, r_hi = oracle.embed_rk4(kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps)
        for a, b in [(0, 40), (300, 357), (650, 700), (0, 700), (101, 102)]:
            w_lo, w_hi = oracle.embed_window(kind, p.prm, lambda i0, c: p.box(i0, c), p.n, a, b,
                                             p.nsteps, pl, ph, dt=p.dt)
            assert np.array_equal(w_lo, r_lo[a:b]) and np.array_equal(w_hi, r_hi[a:b])


# ------------------------------------------------------------- Monte Carlo

def test_mc_zero_steps_returns_extreme_draws():
    """With nsteps = 0 on the box [0, 1] the samples are the raw uniform draws."""
    n, m, seed = 10, 7, 20010638
    mn, mx, S = oracle.montecarlo(oracle.CTM, CTM_PRM, np.zeros(n), np.ones(n), nsteps=0, m=m,
                                  seed=seed, return_samples=True)
    U = np.array([[(int(_numpy_block((j // 4, s, 2, 0), (seed, 0))[j % 4]) >> 11) * 2.0 ** -53
                   for j in range(n)] for s in range(m)])
    assert np.array_equal(S, U)
    assert np.array_equal(mn, U.min(axis=0)) and np.array_equal(mx, U.max(axis=0))


def test_mc_min_max_is_numpy_reduction_of_samples():
    p = workloads.small_problem(oracle.RD, 20, 11, 30)
    lo, hi = p.box()
    pl, ph = p.inputs()
    mn, mx, S = oracle.montecarlo(p.kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps, m=50,
                                  seed=3, return_samples=True)
    assert np.array_equal(mn, np.min(S, axis=0)) and np.array_equal(mx, np.max(S, axis=0))


def test_mc_each_sample_is_a_trajectory():
    p = workloads.small_problem(oracle.RD, 12, 12, 20)
    lo, hi = p.box()
    pl, ph = p.inputs()
    seed = 5
    _, _, S = oracle.montecarlo(p.kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps, m=4,
                                seed=seed, s0=3, return_samples=True)
    for k in range(4):
        s = 3 + k
        x0 = np.array([lo[j] + oracle.uniform(seed, s, j) * (hi[j] - lo[j]) for j in range(p.n)])
        u = pl[0] + oracle.uniform(seed, s, p.n) * (ph[0] - pl[0])
        assert np.array_equal(S[k], oracle.f_rk4(p.kind, p.prm, x0, [u], dt=p.dt,
                                                 nsteps=p.nsteps))


def test_mc_prefix_nesting_and_range_split():
    p = workloads.small_problem(oracle.CTM, 16, 13, 50)
    lo, hi = p.box()
    a = oracle.montecarlo(p.kind, p.prm, lo, hi, dt=p.dt, nsteps=p.nsteps, m=40, seed=1)
    b = oracle.montecarlo(p.kind, p.prm, lo, hi, dt=p.dt, nsteps=p.nsteps, m=100, seed=1)
    assert np.all(b[0] <= a[0]) and np.all(b[1] >= a[1])
    c = oracle.montecarlo(p.kind, p.prm, lo, hi, dt=p.dt, nsteps=p.nsteps, m=60, s0=40, seed=1)
    assert np.array_equal(np.minimum(a[0], c[0]), b[0])
    assert np.array_equal(np.maximum(a[1], c[1]), b[1])


def test_mc_sample_count_is_the_union_bound():
    """m is the least integer with 2n exp(-eps m / (2n)) <= delta."""
    for n, eps, delta in [(1, 0.1, 0.05), (64, 0.01, 0.01), (4096, 0.05, 1e-3), (7, 0.3, 0.5)]:
        m = oracle.mc_samples(n, eps, delta)
        bound = lambda mm: 2 * n * np.exp(-eps * mm / (2 * n))
        assert bound(m) <= delta * (1 + 1e-12)
        assert bound(m - 1) > delta * (1 - 1e-9)
    assert oracle.mc_samples(0, 0.1, 0.1) == -1
    assert oracle.mc_samples(4, 0.0, 0.1) == -1
    assert oracle.mc_samples(4, 0.1, 1.0) == -1


def test_mc_probabilistic_guarantee_holds_statistically():
    """n = 2 (a two-cell RD chain): a box from m = m(eps, delta) samples leaves
    out at most eps of fresh samples in at least 1 - delta of repetitions."""
    n, eps, delta = 2, 0.1, 0.2
    m = oracle.mc_samples(n, eps, delta)
    prm, lo, hi = (1.0,), np.array([-0.5, 0.2]), np.array([0.5, 0.9])
    pl, ph = [-0.1], [0.1]
    fails, trials = 0, 30
    for t in range(trials):
        mn, mx = oracle.montecarlo(oracle.RD, prm, lo, hi, pl, ph, dt=0.1, nsteps=10, m=m,
                                   seed=100 + t)
        _, _, S = oracle.montecarlo(oracle.RD, prm, lo, hi, pl, ph, dt=0.1, nsteps=10, m=2000,
                                    seed=100 + t, s0=10 ** 6, return_samples=True)
        outside = np.mean(np.any((S < mn) | (S > mx), axis=1))
        fails += outside > eps
    # P(fails >= 15 | p <= 0.2, 30 trials) < 1e-4
    assert fails < 15


# ------------------------------------------------------------ growth bound

def test_growth_bound_equals_embedding_on_cooperative_linear_chain():
    """For x' = A x + b u with A Metzler, the embedding's center and half-width
    obey c' = A c + b u*, r' = A r + |b| [u], which is the growth bound with
    C = A: both methods give the same box (Sec. 2.1)."""
    rng = np.random.default_rng(14)
    n = 30
    coef = (0.4, -1.3, 0.25, -0.7)
    lo = rng.uniform(-1, 1, n)
    hi = lo + rng.uniform(0, 0.4, n)
    pl, ph = [-0.2], [0.3]
    g = oracle.growth_bound(oracle.LIN3, coef, lo, hi, pl, ph, dt=0.05, nsteps=60)
    m = oracle.embed_rk4(oracle.LIN3, coef, lo, hi, pl, ph, dt=0.05, nsteps=60)
    np.testing.assert_allclose(g[0], m[0], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g[1], m[1], rtol=1e-12, atol=1e-13)


def test_growth_bound_radius_exact_rational():
    """The half-width follows RK4 of r' = C r + |b| [u] exactly (R(hC), S(hC))."""
    n, coef = 4, (-0.5, -1.0, 0.75, -2.0)
    lo = [0.5, -1.0, 0.25, 1.5]
    hi = [0.75, -0.5, 1.25, 1.625]
    pl, ph = [-0.25], [0.5]
    h, N = 0.0625, 5
    C = cf.tridiag(n, 0.5, -1.0, 0.75)
    half_u = Fraction(1, 2) * (Fraction(0.5) - Fraction(-0.25))
    r0 = [(Fraction(b) - Fraction(a)) / 2 for a, b in zip(lo, hi)]
    r1 = cf.rk4_linear_exact(C, [Fraction(2) * half_u] * n, r0, h, N)
    c1 = cf.rk4_linear_exact(cf.tridiag(n, -0.5, -1.0, 0.75),
                             [Fraction(-2) * (Fraction(-0.25) + Fraction(0.5)) / 2] * n,
                             [(Fraction(a) + Fraction(b)) / 2 for a, b in zip(lo, hi)], h, N)
    g_lo, g_hi = oracle.growth_bound(oracle.LIN3, coef, lo, hi, pl, ph, dt=h, nsteps=N)
    np.testing.assert_allclose(g_hi - g_lo, 2 * cf.to_float(r1), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose((g_hi + g_lo) / 2, cf.to_float(c1), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", [oracle.CTM, oracle.RD])
def test_contraction_matrix_bounds_the_jacobian(kind):
    """C_ii >= J_ii and C_ij >= |J_ij| at random states (central differences)."""
    prm = CTM_PRM if kind == oracle.CTM else (1.0,)
    sub, diag, sup, _ = oracle.contraction_matrix(kind, prm)
    rng = np.random.default_rng(15)
    n, eps = 12, 1e-6
    for trial in range(30):
        y = rng.uniform(0, 40, n) if kind == oracle.CTM else rng.uniform(-2, 2, n)
        p = None if kind == oracle.CTM else [0.05]
        for j in range(n):
            e = np.zeros(n)
            e[j] = eps
            col = (oracle.rhs(kind, prm, y + e, p, use_f=True)
                   - oracle.rhs(kind, prm, y - e, p, use_f=True)) / (2 * eps)
            assert col[j] <= diag + 1e-6
            if j > 0:
                assert abs(col[j - 1]) <= sup + 1e-6      # d f_{j-1} / d y_j
            if j < n - 1:
                assert abs(col[j + 1]) <= sub + 1e-6      # d f_{j+1} / d y_j


@pytest.mark.parametrize("kind", [oracle.CTM, oracle.RD])
def test_growth_bound_contains_embedding_and_samples(kind):
    p = workloads.small_problem(kind, 48, 16, 80)
    lo, hi = p.box()
    pl, ph = p.inputs()
    g = oracle.growth_bound(kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps)
    m = oracle.embed_rk4(kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps)
    assert np.all(g[0] <= m[0] + 1e-12) and np.all(g[1] >= m[1] - 1e-12)
    _, _, S = oracle.montecarlo(kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps, m=200,
                                seed=4, return_samples=True)
    assert np.all(S >= g[0]) and np.all(S <= g[1])


def test_growth_bound_degenerate_box_is_the_trajectory():
    p = workloads.small_problem(oracle.CTM, 25, 17, 40)
    lo, _ = p.box()
    g = oracle.growth_bound(p.kind, p.prm, lo, lo, dt=p.dt, nsteps=p.nsteps)
    traj = oracle.f_rk4(p.kind, p.prm, lo, None, dt=p.dt, nsteps=p.nsteps)
    assert np.array_equal(g[0], traj) and np.array_equal(g[1], traj)


def test_growth_bound_window_is_bitwise_whole_chain():
    p = workloads.small_problem(oracle.RD, 600, 18, 20)
    lo, hi = p.box()
    pl, ph = p.inputs()
    full = oracle.growth_bound(p.kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=p.nsteps)
    a, b = 250, 300
    r = 4 * p.nsteps
    w = oracle.growth_bound(p.kind, p.prm, lo[a - r:b + r], hi[a - r:b + r], pl, ph, dt=p.dt,
                            nsteps=p.nsteps, n_total=p.n, g0=a - r)
    assert np.array_equal(w[0][r:r + b - a], full[0][a:b])
    assert np.array_equal(w[1][r:r + b - a], full[1][a:b])


# ------------------------------------------------------- 3-D heat pins

def _heat_A_by_edges(nx, ny, nz, a):
    """The heat system's matrix built from its graph: one entry pair per edge
    between face-adjacent cells, plus the loss of each cell on the open face
    x = nx - 1 (Sec. 5, heat diffusion: insulated but for one face)."""
    n = nx * ny * nz
    A = cf.mat(n)
    cells = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    idx = {c: t for t, c in enumerate(cells)}
    for (i, j, k), p in idx.items():
        for di, dj, dk in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
            q = idx.get((i + di, j + dj, k + dk))
            if q is not None:      # the edge p -- q: heat flows both ways
                A[p][q] += a
                A[q][p] += a
                A[p][p] -= a
                A[q][q] -= a
        if i == nx - 1:
            A[p][p] -= a
    return A


@pytest.mark.parametrize("dims", [(3, 2, 2), (2, 3, 1), (1, 1, 3), (1, 2, 1)])
def test_heat3d_trajectory_exact_rational(dims):
    """RK4 of the heat grid equals R(hA)^N x0 with A built edge by edge."""
    nx, ny, nz = dims
    alpha, dx, h, N = 0.375, 0.5, 0.0625, 3
    a = Fraction(alpha) / (Fraction(dx) ** 2)
    n = nx * ny * nz
    x0 = [Fraction(((7 * t) % 11) - 5, 4) for t in range(n)]
    A = _heat_A_by_edges(nx, ny, nz, a)
    exact = cf.to_float(cf.rk4_linear_exact(A, [0] * n, x0, h, N))
    prm = oracle.heat3d_prm(nx, ny, nz, alpha, dx)
    got = oracle.f_rk4(oracle.HEAT3D, prm, [float(v) for v in x0], None, dt=h, nsteps=N)
    np.testing.assert_allclose(got, exact, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("modes", [(0, 0, 0), (1, 2, 1), (2, 0, 3), (4, 3, 0)])
def test_heat3d_cosine_mode_decays_by_stability_polynomial(modes):
    """Separable eigenvectors of the grid operator: cos((i + 1/2) t) along x
    with t = (m + 1/2) pi / (nx + 1/2) (insulated at x = 0, zero outside
    x = nx - 1), cos((j + 1/2) m pi / ny) along the insulated y and z.  The
    eigenvalue is alpha / dx^2 times the sum of 2 cos(t) - 2 over the axes,
    and RK4 multiplies the mode by R(dt lambda) per step."""
    nx, ny, nz = 9, 7, 5
    alpha, dx, dt, N = 0.02, 0.1, 0.05, 30
    mx, my, mz = modes
    tx = (mx + 0.5) * np.pi / (nx + 0.5)
    ty, tz = my * np.pi / ny, mz * np.pi / nz
    i, j, k = np.arange(nx), np.arange(ny), np.arange(nz)
    u0 = (np.cos((k[:, None, None] + 0.5) * tz) * np.cos((j[None, :, None] + 0.5) * ty)
          * np.cos((i[None, None, :] + 0.5) * tx)).ravel()
    lam = alpha / dx ** 2 * ((2 * np.cos(tx) - 2) + (2 * np.cos(ty) - 2) + (2 * np.cos(tz) - 2))
    prm = oracle.heat3d_prm(nx, ny, nz, alpha, dx)
    got = oracle.f_rk4(oracle.HEAT3D, prm, u0, None, dt=dt, nsteps=N)
    np.testing.assert_allclose(got, cf.rk4_stability(lam * dt) ** N * u0, rtol=0,
                               atol=1e-13 * np.max(np.abs(u0)))


def test_heat3d_heat_leaves_only_through_the_open_face():
    """Summed over the grid, the flows between cells cancel: d/dt of the total
    heat is alpha / dx^2 times minus the sum of u over the face x = nx - 1."""
    nx, ny, nz, alpha, dx = 6, 5, 4, 0.3, 0.25
    rng = np.random.default_rng(21)
    u = rng.uniform(0.0, 1.0, nx * ny * nz)
    f = oracle.rhs(oracle.HEAT3D, oracle.heat3d_prm(nx, ny, nz, alpha, dx), u, use_f=True)
    face = u.reshape(nz, ny, nx)[:, :, nx - 1].sum()
    assert abs(f.sum() - (-alpha / dx ** 2 * face)) < 1e-11 * alpha / dx ** 2 * u.size


def test_heat3d_embedding_is_two_trajectories_and_ordered():
    """Off-diagonal entries alpha / dx^2 >= 0: cooperative, d = f, so the
    embedding is RK4 of f from each corner, and stays ordered."""
    nx, ny, nz = 8, 6, 5
    prm = oracle.heat3d_prm(nx, ny, nz, 0.01, 0.1)
    rng = np.random.default_rng(22)
    lo = rng.uniform(0.0, 1.0, nx * ny * nz)
    hi = lo + rng.uniform(0.0, 0.2, lo.size)
    r_lo, r_hi = oracle.embed_rk4(oracle.HEAT3D, prm, lo, hi, dt=0.05, nsteps=40)
    assert np.array_equal(r_lo, oracle.f_rk4(oracle.HEAT3D, prm, lo, None, dt=0.05, nsteps=40))
    assert np.array_equal(r_hi, oracle.f_rk4(oracle.HEAT3D, prm, hi, None, dt=0.05, nsteps=40))
    assert np.all(r_lo <= r_hi)


def test_heat3d_growth_bound_equals_embedding():
    """Linear and Metzler: the growth bound with C = A is the embedding's box."""
    nx, ny, nz = 7, 4, 6
    prm = oracle.heat3d_prm(nx, ny, nz, 0.01, 0.1)
    rng = np.random.default_rng(23)
    lo = rng.uniform(-1.0, 1.0, nx * ny * nz)
    hi = lo + rng.uniform(0.0, 0.5, lo.size)
    g = oracle.growth_bound(oracle.HEAT3D, prm, lo, hi, dt=0.05, nsteps=30)
    m = oracle.embed_rk4(oracle.HEAT3D, prm, lo, hi, dt=0.05, nsteps=30)
    np.testing.assert_allclose(g[0], m[0], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g[1], m[1], rtol=1e-12, atol=1e-13)


def test_heat3d_window_is_bitwise_whole_grid():
    nx, ny, nz, nsteps = 30, 26, 22, 2
    prm = oracle.heat3d_prm(nx, ny, nz, 0.01, 0.1)
    rng = np.random.default_rng(24)
    lo = rng.uniform(0.0, 1.0, nx * ny * nz)
    hi = lo + 0.1
    full = oracle.embed_rk4(oracle.HEAT3D, prm, lo, hi, dt=0.05, nsteps=nsteps)
    L, H = lo.reshape(nz, ny, nx), hi.reshape(nz, ny, nx)

    def box(o, d):
        s = (slice(o[2], o[2] + d[2]), slice(o[1], o[1] + d[1]), slice(o[0], o[0] + d[0]))
        return L[s].ravel(), H[s].ravel()

    for a, b in [((0, 0, 0), (5, 4, 3)), ((12, 9, 10), (20, 15, 13)), ((25, 20, 17), (30, 26, 22))]:
        w_lo, w_hi = oracle.heat3d_window(prm, box, a, b, nsteps, dt=0.05)
        s = (slice(a[2], b[2]), slice(a[1], b[1]), slice(a[0], b[0]))
        assert np.array_equal(w_lo, full[0].reshape(nz, ny, nx)[s])
        assert np.array_equal(w_hi, full[1].reshape(nz, ny, nx)[s])
