"""The seeded input generators: recipes restated with numpy from the same
uniform draws (which are pinned against numpy's Philox elsewhere), window
consistency, and the heat corner's geometry."""
import numpy as np
import pytest

import workloads


def test_ctm_recipe_from_uniforms():
    n, seed = 1000, 77
    u0 = workloads.uniform(seed, 0, 0, n)
    u1 = workloads.uniform(seed, 1, 0, n)
    lo, hi = workloads.box(workloads.CTM_RANDW, (12.0, 2.0), seed, n)
    assert np.array_equal(lo, 12.0 + 12.0 * u0)
    assert np.array_equal(hi, lo + 2.0 * u1)


def test_heat_corner_recipe_from_uniforms():
    nx, ny, nz, seed = 9, 7, 6, 78
    p = workloads.heat3d_problem(nx, ny, nz, seed, 1)
    lo, hi = p.box()
    u0 = workloads.uniform(seed, 0, 0, p.n).reshape(nz, ny, nx)
    u1 = workloads.uniform(seed, 1, 0, p.n).reshape(nz, ny, nx)
    c, b, a = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    heated = (a < 0.5 * nx) & (b < 0.5 * ny) & (c < 0.5 * nz)
    f, T, hw, cw = workloads.HEAT_BOX
    exp_lo = np.where(heated, T - hw * u0, 0.0)
    exp_hi = np.where(heated, T + hw * u1, cw * u1)
    assert np.array_equal(lo.reshape(nz, ny, nx), exp_lo)
    assert np.array_equal(hi.reshape(nz, ny, nx), exp_hi)
    assert heated.sum() == 5 * 4 * 3 and np.all(lo <= hi)


@pytest.mark.parametrize("recipe,prm", [(workloads.CTM_RANDW, (12.0, 2.0)),
                                        (workloads.SIN, (0.02,)),
                                        (workloads.HEAT_CORNER, (10.0, 10.0, 10.0) +
                                         workloads.HEAT_BOX)])
def test_windows_are_slices_of_the_whole(recipe, prm):
    n, seed = 1000, 79
    lo, hi = workloads.box(recipe, prm, seed, n)
    for i0, cnt in ((0, 1), (3, 17), (401, 333), (999, 1)):
        wl, wh = workloads.box(recipe, prm, seed, n, i0, cnt)
        assert np.array_equal(wl, lo[i0:i0 + cnt]) and np.array_equal(wh, hi[i0:i0 + cnt])
    l32, h32 = workloads.box(recipe, prm, seed, n, dtype=np.float32)
    assert np.array_equal(l32, lo.astype(np.float32)) and np.array_equal(h32, hi.astype(np.float32))


def test_heat_case_study_parameters():
    p = workloads.heat3d_1000_f64()
    assert p.n == 10 ** 9 and p.nsteps == 1000 and p.dt == 0.02
    nx, ny, nz, alpha, dx = p.prm
    assert (nx, ny, nz) == (1000.0, 1000.0, 1000.0) and dx == 1e-3
    # RK4 stays stable: spectral radius of the grid operator times dt below
    # the stability interval's end on the negative axis (about 2.785)
    assert 12 * alpha / dx ** 2 * p.dt < 2.785
