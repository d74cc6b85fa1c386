"""GPU parity of the 3-D heat grid (heat diffusion case study, Sec. 5) against
the FP64 oracle: the embedding (Algorithm 3 with the RK4 of Algorithm 1) and
the growth bound (Algorithm 2), at small sizes element by element, and at
the case study's full size (1000^3 cells, 1000 steps) through sampled
windows and the closed-form decay of a separable cosine mode."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import RTOL, assert_rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2001_10635_amd")

ROWS = {np.float64: [2, 4, 5, 3], np.float32: [2, 4, 3, 8]}
GRIDS = [(1, 1, 1), (2, 1, 1), (1, 3, 1), (1, 1, 5), (3, 2, 2), (7, 5, 4), (56, 24, 6),
         (57, 25, 7), (64, 32, 14), (70, 45, 13), (113, 50, 21), (5, 130, 9), (200, 3, 30)]


@pytest.fixture(scope="module")
def rc():
    r = R.Reach(0)
    yield r
    r.close()


@pytest.fixture(autouse=True)
def _reset(rc):
    rc.set_option("heat.P", 0)
    yield
    rc.set_option("heat.P", 0)


def heat_case(grid, dtype, seed, alpha=0.01, dx=0.1, dt=0.05):
    nx, ny, nz = grid
    p = workloads.heat3d_problem(nx, ny, nz, seed, 0, dtype=dtype, dt=dt, alpha=alpha, dx=dx)
    lo, hi = p.box()
    return list(p.prm), lo, hi, dt


def run_embed(rc, prm, lo, hi, dt, nsteps, **kw):
    r_lo, r_hi = rc.embed(R.REACH_HEAT3D, prm, to_dev(lo), to_dev(hi), dt, nsteps, **kw)
    st = rc.sync()
    return to_host(r_lo), to_host(r_hi), st


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: "x".join(map(str, g)))
def test_heat3d_embed_matches_oracle(rc, grid, dtype):
    prm, lo, hi, dt = heat_case(grid, dtype, seed=sum(grid))
    rt = RTOL[np.dtype(dtype)]
    for nsteps in (1, 5):
        o_lo, o_hi = oracle.embed_rk4(oracle.HEAT3D, prm, lo.astype(np.float64),
                                      hi.astype(np.float64), dt=dt, nsteps=nsteps)
        for P in ROWS[dtype]:
            rc.set_option("heat.P", P)
            say(f"heat3d {grid} {np.dtype(dtype).name} P={P} steps={nsteps}")
            g_lo, g_hi, st = run_embed(rc, prm, lo, hi, dt, nsteps)
            assert st == R.REACH_OK
            assert_rel(g_lo, o_lo, rt, f"lower P={P}")
            assert_rel(g_hi, o_hi, rt, f"upper P={P}")


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_heat3d_tile_shape_invariance_is_bitwise(rc, dtype):
    """Each cell sums the same operands in the same order whatever the tile."""
    prm, lo, hi, dt = heat_case((150, 77, 19), dtype, seed=41)
    outs = []
    for P in ROWS[dtype]:
        rc.set_option("heat.P", P)
        say(f"heat3d shape P={P}")
        outs.append(run_embed(rc, prm, lo, hi, dt, 9)[:2])
    for a, b in outs[1:]:
        assert np.array_equal(a, outs[0][0]) and np.array_equal(b, outs[0][1])


def test_heat3d_resume_alias_and_zero_steps(rc):
    prm, lo, hi, dt = heat_case((90, 40, 11), np.float64, seed=42)
    say("heat3d resume")
    a_lo, a_hi, _ = run_embed(rc, prm, lo, hi, dt, 7)
    b_lo, b_hi, _ = run_embed(rc, prm, lo, hi, dt, 3)
    c_lo, c_hi, _ = run_embed(rc, prm, b_lo, b_hi, dt, 4)
    assert np.array_equal(a_lo, c_lo) and np.array_equal(a_hi, c_hi)
    say("heat3d in place")
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    rc.embed(R.REACH_HEAT3D, prm, x_lo, x_hi, dt, 7, r_lo=x_lo, r_hi=x_hi)
    assert rc.sync() == R.REACH_OK
    assert np.array_equal(to_host(x_lo), a_lo) and np.array_equal(to_host(x_hi), a_hi)
    say("heat3d swapped aliases, odd and even step counts")
    for nsteps in (1, 2, 5):
        x_lo, x_hi = to_dev(lo), to_dev(hi)
        r_lo, r_hi = rc.embed(R.REACH_HEAT3D, prm, x_lo, x_hi, dt, nsteps, r_lo=x_hi, r_hi=x_lo)
        assert rc.sync() == R.REACH_OK
        o_lo, o_hi, _ = run_embed(rc, prm, lo, hi, dt, nsteps)
        assert np.array_equal(to_host(r_lo), o_lo) and np.array_equal(to_host(r_hi), o_hi)
    z_lo, z_hi, st = run_embed(rc, prm, lo, hi, dt, 0)
    assert st == R.REACH_OK and np.array_equal(z_lo, lo) and np.array_equal(z_hi, hi)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("grid", [(1, 1, 1), (3, 2, 2), (57, 25, 7), (113, 50, 21)],
                         ids=lambda g: "x".join(map(str, g)))
def test_heat3d_growth_bound_matches_oracle(rc, grid, dtype):
    prm, lo, hi, dt = heat_case(grid, dtype, seed=7 + sum(grid))
    say(f"heat3d gb {grid} {np.dtype(dtype).name}")
    for nsteps in (0, 1, 6):
        g_lo, g_hi = rc.growth_bound(R.REACH_HEAT3D, prm, to_dev(lo), to_dev(hi), dt, nsteps)
        assert rc.sync() == R.REACH_OK
        o_lo, o_hi = oracle.growth_bound(oracle.HEAT3D, prm, lo.astype(np.float64),
                                         hi.astype(np.float64), dt=dt, nsteps=nsteps)
        rt = RTOL[np.dtype(dtype)]
        assert_rel(to_host(g_lo), o_lo, rt, "gb lower")
        assert_rel(to_host(g_hi), o_hi, rt, "gb upper")


def test_heat3d_rejected_where_unsupported(rc):
    prm, lo, hi, dt = heat_case((4, 3, 2), np.float64, seed=1)
    x = to_dev(lo)
    n = x.numel()
    lib = R.lib()

    def embed(sys, ws=None, nb=0):
        return lib.reach_embed_rk4(rc.ctx, R.ctypes.byref(sys), R.REACH_F64, x.data_ptr(),
                                   x.data_ptr(), None, None, 0.0, dt, 1, x.data_ptr(),
                                   x.data_ptr(), ws, nb, None)

    say("heat3d invalid systems")
    assert embed(R.make_system(R.REACH_HEAT3D, n + 1, prm)) == R.REACH_E_INVAL
    assert embed(R.make_system(R.REACH_HEAT3D, n, [4.5, 3, 2, 0.01, 0.1])) == R.REACH_E_INVAL
    assert embed(R.make_system(R.REACH_HEAT3D, n, [4, 3, 2, -0.01, 0.1])) == R.REACH_E_INVAL
    assert embed(R.make_system(R.REACH_HEAT3D, n, [4, 3, 2, 0.01, 0.0])) == R.REACH_E_INVAL
    assert embed(R.make_system(R.REACH_HEAT3D, n, prm, 1)) == R.REACH_E_UNSUPPORTED
    sys = R.make_system(R.REACH_HEAT3D, n, prm)
    st = lib.reach_montecarlo(rc.ctx, R.ctypes.byref(sys), R.REACH_F64, x.data_ptr(),
                              x.data_ptr(), None, None, 0.0, dt, 1, 16, 1, x.data_ptr(),
                              x.data_ptr(), x.data_ptr(), 1 << 20, None)
    assert st == R.REACH_E_UNSUPPORTED
    with pytest.raises(R.ReachError):
        rc.set_option("heat.P", 7)


def _heat_1000():
    return workloads.heat3d_1000_f64()


@pytest.fixture(scope="module")
def big_box():
    p = _heat_1000()
    say("heat3d 1000^3 box generation (host)")
    lo = np.empty(p.n, dtype=np.float64)
    hi = np.empty(p.n, dtype=np.float64)
    p.box(out=(lo, hi))
    return p, lo, hi


def test_heat3d_1000_windows_match_oracle(rc, big_box):
    """The case study's grid and box, eight steps (eight launches of the
    one-step kernel, ping-ponged), sampled 8^3 blocks checked against oracle
    runs on their light cones (four cells per stage and face)."""
    p, lo, hi = big_box
    nx = ny = nz = 1000
    steps = 8
    say(f"heat3d 1000^3 {steps} steps")
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    r_lo, r_hi = rc.embed(R.REACH_HEAT3D, list(p.prm), x_lo, x_hi, p.dt, steps)
    assert rc.sync() == R.REACH_OK
    del x_lo, x_hi
    L, H = lo.reshape(nz, ny, nx), hi.reshape(nz, ny, nx)
    g_lo, g_hi = r_lo.view(nz, ny, nx), r_hi.view(nz, ny, nx)

    def box(o, d):
        s = (slice(o[2], o[2] + d[2]), slice(o[1], o[1] + d[1]), slice(o[0], o[0] + d[0]))
        return L[s].ravel(), H[s].ravel()

    rng = np.random.default_rng(5)
    corners = [(0, 0, 0), (992, 992, 992), (992, 0, 500), (0, 992, 7), (496, 496, 496),
               (52, 20, 0), (55, 23, 999 - 7)]
    corners += [tuple(int(v) for v in rng.integers(0, 993, 3)) for _ in range(5)]
    for a in corners:
        b = tuple(v + 8 for v in a)
        o_lo, o_hi = oracle.heat3d_window(list(p.prm), box, a, b, steps, dt=p.dt)
        s = (slice(a[2], b[2]), slice(a[1], b[1]), slice(a[0], b[0]))
        assert_rel(to_host(g_lo[s]), o_lo, 1e-12, f"lower block {a}")
        assert_rel(to_host(g_hi[s]), o_hi, 1e-12, f"upper block {a}")


def test_heat3d_1000_full_run_cosine_mode(rc):
    """1000 steps on the 1000^3 grid from a separable cosine mode (an
    eigenvector of the grid operator with its boundary faces, see the oracle
    pins): every cell decays by R(dt lambda)^1000, R the RK4 polynomial."""
    nx = ny = nz = 1000
    p = _heat_1000()
    alpha, dx = p.prm[3], p.prm[4]
    mx, my, mz = 7, 3, 5
    tx = (mx + 0.5) * np.pi / (nx + 0.5)
    ty, tz = my * np.pi / ny, mz * np.pi / nz
    cx = torch.cos((torch.arange(nx, dtype=torch.float64) + 0.5) * tx).cuda()
    cy = torch.cos((torch.arange(ny, dtype=torch.float64) + 0.5) * ty).cuda()
    cz = torch.cos((torch.arange(nz, dtype=torch.float64) + 0.5) * tz).cuda()
    mode = (cz[:, None, None] * cy[None, :, None] * cx[None, None, :]).reshape(-1)
    # the lowest mode is positive everywhere, so [mode, mode + 2 mode0] is a box
    t0x = 0.5 * np.pi / (nx + 0.5)
    c0 = torch.cos((torch.arange(nx, dtype=torch.float64) + 0.5) * t0x).cuda()
    mode0 = c0.repeat(ny * nz)

    def decay(lam):
        z = lam * p.dt
        return (1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0) ** p.nsteps

    a = alpha / dx ** 2
    f1 = decay(a * ((2 * np.cos(tx) - 2) + (2 * np.cos(ty) - 2) + (2 * np.cos(tz) - 2)))
    f0 = decay(a * (2 * np.cos(t0x) - 2))
    say("heat3d 1000^3 full run (1000 steps) on cosine modes")
    x_lo = mode
    x_hi = mode + 2.0 * mode0
    r_lo, r_hi = rc.embed(R.REACH_HEAT3D, list(p.prm), x_lo, x_hi, p.dt, p.nsteps)
    assert rc.sync() == R.REACH_OK
    ref_lo = f1 * mode
    ref_hi = f1 * mode + 2.0 * f0 * mode0
    err_lo = torch.max(torch.abs(r_lo - ref_lo) / torch.clamp(torch.abs(ref_lo), min=1.0)).item()
    err_hi = torch.max(torch.abs(r_hi - ref_hi) / torch.clamp(torch.abs(ref_hi), min=1.0)).item()
    say(f"heat3d cosine mode: rel err lower {err_lo:.2e} upper {err_hi:.2e}")
    assert 0.5 < f1 < 0.95 and 0.99 < f0 < 1.0
    assert err_lo <= 1e-12 and err_hi <= 1e-12, (err_lo, err_hi, f1, f0)
