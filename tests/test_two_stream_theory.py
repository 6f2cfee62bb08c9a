"""The two-stream dispersion root finder against the paper's closed-form
maximum growth rate and its wavenumber, and the reference's whole loop
(Faraday, particle step, Ampere) against that theory (Sec. 5.1.1)."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.two_stream_theory import linear_stage_rate, mode_power, setup, two_stream_growth


def test_dispersion_root_finder_matches_the_closed_form_maximum():
    wp, ub = 0.025, 0.5
    gb = np.sqrt(1 + ub * ub)
    vb = ub / gb
    kmax = np.sqrt(3) * wp / ((2 * gb) ** 1.5 * vb)
    assert two_stream_growth(kmax, wp, ub) == pytest.approx(wp / (2 * gb) ** 1.5, rel=1e-9)
    ks = np.linspace(0.2, 3, 200) * kmax
    assert max(two_stream_growth(k, wp, ub) for k in ks) <= wp / (2 * gb) ** 1.5 * (1 + 1e-9)


def test_reference_loop_grows_the_two_stream_mode_at_the_theoretical_rate():
    """Seeded mode 5 of a 256-cell box of 25.6 skin depths (the box's fastest
    mode, Gamma = 0.298 wp) on the reference's whole loop, 35 / wp."""
    wp, ub, mode = 0.1, 0.5, 5
    grid, species = setup(nx=256, ny=2, ppc=32, wp=wp, ub=ub, mode=mode)
    g = O.make_grid("cart", 2, grid["n"], grid["lo"], grid["hi"])
    dt = O.dt_from_cfl(g, 0.45)
    EB = np.zeros((6,) + O.padded_shape(g))
    prof, ts = [], []
    for s in range(int(35 / wp / dt)):
        if s % 10 == 0:
            prof.append(EB[0, 0, 2:4, 2:258].mean(0).copy())
            ts.append(s * dt * wp)
        EB = O.faraday(g, EB, 0.5 * dt)
        species, J = O.run(g, dt, 1, EB, species)
        EB = O.faraday(g, EB, 0.5 * dt)
        EB = O.ampere(g, EB, J, dt, 4 * np.pi)
    rate, win = linear_stage_rate(np.array(ts), np.log(mode_power(prof, mode)))
    theory = two_stream_growth(2 * np.pi * mode / 256, wp, ub) / wp
    assert rate == pytest.approx(theory, rel=0.05), (rate, theory, win)
