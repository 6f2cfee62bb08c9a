"""Physics validation of the whole loop on the GPU (Sec. 5.1.1): the
relativistic two-stream instability of two cold counter-streaming electron
beams over a neutralising static background, and the Weibel (filamentation)
instability of the same beams streaming along z across a 2D x-y box.  One Fourier mode of the box
(the fastest it holds) is seeded; in its linear stage its amplitude grows
at the rate given by the roots of the dispersion relation (eq.
two_stream_dispersion), 0.298 wp for beams of four-velocity +-0.5.  The box
is 2D, a few cells across (the instability is longitudinal along x), and
holds 25.6 skin depths, as in the paper's 1D run; the reference's loop is
held to the same theory in tests/test_two_stream_theory.py.

Units: fields in B0, lengths in rho0 = 1 code length (unit cells), c = 1;
with the coupling 4 pi of Ampere's law a species of weight density n and
q = m = 1 has wp^2 = 4 pi n."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_17710_amd import workloads as W
from tests import weibel_theory as WT
from tests.two_stream_theory import linear_stage_rate, mode_power, setup, two_stream_growth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_two_stream_growth_rate(prec):
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[validation] two-stream {prec}", flush=True)
    nx, ny, wp, ub, mode = 256, 4, 0.1, 0.5, 5
    grid, species = setup(nx=nx, ny=ny, ppc=64, wp=wp, ub=ub, mode=mode)
    wl = W.Workload(name="two_stream", geom="cart", dim=2, n=grid["n"], lo=grid["lo"],
                    hi=grid["hi"], steps=0, sort_every=20, seed=0)
    wl.species = species
    wl.fields_tetrad = np.zeros((6, 1, ny, nx))
    wl.fields_includes_ghosts = 0
    ctx = P.from_workload(wl, prec=prec)
    g = O.make_grid("cart", 2, wl.n, wl.lo, wl.hi)
    dt = O.dt_from_cfl(g, wl.cfl)
    every = 10
    prof, ts = [], []
    for n in range(0, int(35 / wp / dt), every):
        # E_x along the box, averaged across it
        prof.append(ctx.fields()[0, 0, 2:2 + ny, 2:2 + nx].double().mean(dim=0).cpu().numpy())
        ts.append(n * dt * wp)
        ctx.step_full(dt, every, 0, 4 * np.pi)
    torch.cuda.synchronize()
    rate, win = linear_stage_rate(np.array(ts), np.log(mode_power(prof, mode)))
    theory = two_stream_growth(2 * np.pi * mode / nx, wp, ub) / wp
    gb = np.sqrt(1 + ub * ub)
    print(f"  mode {mode}: Gamma/wp {rate:.4f} against {theory:.4f} (Gamma_max/wp "
          f"{1 / (2 * gb) ** 1.5:.4f}), fit over wp t in [{win[0]:.1f}, {win[1]:.1f}]",
          flush=True)
    assert rate == pytest.approx(theory, rel=0.05)


def _weibel_reference_rate(wp, ub, mode, nx, ny, ppc, amp, steps, every):
    """The same seeded run on the reference's whole loop (FP64)."""
    grid, species = WT.setup(nx=nx, ny=ny, ppc=ppc, wp=wp, ub=ub, temp=1e-6)
    g = O.make_grid("cart", 2, grid["n"], grid["lo"], grid["hi"])
    dt = O.dt_from_cfl(g, 0.45)
    EB = WT.seed_by(nx, ny, mode, amp, pad=2)
    prof, ts = [], []
    for s in range(steps):
        if s % every == 0:
            prof.append(EB[4, 0, 2:2 + ny, 2:2 + nx].mean(0).copy())
            ts.append(s * dt * wp)
        EB = O.faraday(g, EB, 0.5 * dt)
        species, J = O.run(g, dt, 1, EB, species)
        EB = O.faraday(g, EB, 0.5 * dt)
        EB = O.ampere(g, EB, J, dt, 4 * np.pi)
    return WT.fixed_window_rate(ts, np.log(mode_power(prof, mode)))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_weibel_growth_rate(prec):
    """Mode 8 of a 128-cell box of 12.8 skin depths (k = 3.93 wp / c: rate
    0.411 wp by the linear theory, within 3 % of the paper's maximum
    v_b wp / sqrt(gamma_b)), seeded in B_y over a quiet start (the beams on
    the same positions with opposite four-velocities), 12 / wp of the whole
    loop; the rate over wp t in [5, 11] within 5 % of the theory and within
    1 % (FP64) or 3 % (FP32) of the reference's loop on the same run."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[validation] Weibel {prec}", flush=True)
    nx, ny, ppc, wp, ub, mode, amp = 128, 2, 32, 0.1, 0.5, 8, 1e-6
    grid, species = WT.setup(nx=nx, ny=ny, ppc=ppc, wp=wp, ub=ub, temp=1e-6)
    wl = W.Workload(name="weibel", geom="cart", dim=2, n=grid["n"], lo=grid["lo"],
                    hi=grid["hi"], steps=0, sort_every=20, seed=0)
    wl.species = species
    wl.fields_tetrad = WT.seed_by(nx, ny, mode, amp)
    wl.fields_includes_ghosts = 0
    ctx = P.from_workload(wl, prec=prec)
    g = O.make_grid("cart", 2, wl.n, wl.lo, wl.hi)
    dt = O.dt_from_cfl(g, wl.cfl)
    every = 5
    steps = int(12 / wp / dt) + 1
    prof, ts = [], []
    for n in range(0, steps, every):
        # B_y along the box, averaged across it
        prof.append(ctx.fields()[4, 0, 2:2 + ny, 2:2 + nx].double().mean(dim=0).cpu().numpy())
        ts.append(n * dt * wp)
        ctx.step_full(dt, every, 0, 4 * np.pi)
    torch.cuda.synchronize()
    rate = WT.fixed_window_rate(ts, np.log(mode_power(prof, mode)))
    ref = _weibel_reference_rate(wp, ub, mode, nx, ny, ppc, amp, steps, every)
    theory = WT.filamentation_growth(2 * np.pi * mode / nx, wp, ub) / wp
    print(f"  mode {mode}: Gamma/wp {rate:.4f}, reference loop {ref:.4f}, theory {theory:.4f} "
          f"(Gamma_max/wp {WT.weibel_max_rate(wp, ub) / wp:.4f})", flush=True)
    assert rate == pytest.approx(theory, rel=0.05)
    assert rate == pytest.approx(ref, rel=0.01 if prec == "f64" else 0.03)
    assert ctx.device_errors() == 0
