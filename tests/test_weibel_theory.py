"""The filamentation (Weibel) growth rate of the linear theory against the
paper's maximum rate and against its own small-k limit, and the reference's
whole loop (Faraday, particle step, Ampere) against that theory on a seeded
mode (Sec. 5.1.1)."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.two_stream_theory import mode_power
from tests.weibel_theory import (filamentation_growth, fixed_window_rate, seed_by, setup,
                                 weibel_max_rate)


def test_filamentation_rate_limits():
    """Gamma(k) grows with k towards the paper's v_b wp / sqrt(gamma_b); for
    k << wp / gamma^(3/2) the magnetic term balances the longitudinal
    inertia and Gamma -> k v_b gamma_b."""
    wp, ub = 0.1, 0.5
    gb = np.sqrt(1 + ub * ub)
    vb = ub / gb
    gmax = weibel_max_rate(wp, ub)
    assert gmax == pytest.approx(0.42294850537622564 * wp, rel=1e-12)
    assert filamentation_growth(1e5 * wp, wp, ub) == pytest.approx(gmax, rel=1e-8)
    ks = np.geomspace(1e-3, 1e3, 200) * wp
    g = np.array([filamentation_growth(k, wp, ub) for k in ks])
    assert np.all(np.diff(g) > 0) and np.all(g < gmax)
    k = 1e-4 * wp
    assert filamentation_growth(k, wp, ub) == pytest.approx(k * vb * gb, rel=1e-6)


def test_reference_loop_grows_the_filamentation_mode_at_the_theoretical_rate():
    """Mode 8 of a 128-cell box of 12.8 skin depths (k = 3.93 wp / c, where
    the rate is 0.411 wp, within 3 % of the paper's maximum), seeded in B_y
    over a quiet start, on the reference's whole loop for 12 / wp; the rate
    over wp t in [5, 11]."""
    wp, ub, mode, nx, ny = 0.1, 0.5, 8, 128, 2
    grid, species = setup(nx=nx, ny=ny, ppc=32, wp=wp, ub=ub, temp=1e-6)
    g = O.make_grid("cart", 2, grid["n"], grid["lo"], grid["hi"])
    dt = O.dt_from_cfl(g, 0.45)
    EB = seed_by(nx, ny, mode, 1e-6, pad=2)
    prof, ts = [], []
    for s in range(int(12 / wp / dt) + 1):
        if s % 5 == 0:
            prof.append(EB[4, 0, 2:2 + ny, 2:2 + nx].mean(0).copy())
            ts.append(s * dt * wp)
        EB = O.faraday(g, EB, 0.5 * dt)
        species, J = O.run(g, dt, 1, EB, species)
        EB = O.faraday(g, EB, 0.5 * dt)
        EB = O.ampere(g, EB, J, dt, 4 * np.pi)
    rate = fixed_window_rate(ts, np.log(mode_power(prof, mode)))
    theory = filamentation_growth(2 * np.pi * mode / nx, wp, ub) / wp
    assert theory == pytest.approx(weibel_max_rate(wp, ub) / wp, rel=0.03)
    assert rate == pytest.approx(theory, rel=0.05), (rate, theory)


def test_quiet_start_setup():
    """The two beams sit on the same positions with opposite four-velocities
    (no current anywhere at the start), stream along +-z at u_b, and their
    weights give wp^2 = 4 pi (weight per unit volume)."""
    wp, ub, nx, ny, ppc = 0.1, 0.5, 16, 2, 8
    grid, (a, b) = setup(nx=nx, ny=ny, ppc=ppc, wp=wp, ub=ub, temp=1e-6)
    np.testing.assert_array_equal(a["cell"], b["cell"])
    np.testing.assert_array_equal(a["offs"], b["offs"])
    np.testing.assert_array_equal(a["u"], -b["u"])
    assert abs(a["u"][:, 2].mean() - ub) < 1e-3 and np.abs(a["u"][:, :2]).max() < 1e-2
    w_total = a["w"].sum() + b["w"].sum()
    assert 4 * np.pi * w_total / (nx * ny) == pytest.approx(wp * wp, rel=1e-12)
    EB = seed_by(nx, ny, 3, 1e-6, pad=2)
    assert np.count_nonzero(EB[[0, 1, 2, 3, 5]]) == 0
    x = np.arange(nx + 4) - 2 + 0.5
    np.testing.assert_allclose(EB[4, 0, 0], 1e-6 * np.sin(2 * np.pi * 3 * x / nx))
