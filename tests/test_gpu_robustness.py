"""Determinism, resume and race checks of the particle step on the GPU, and
the device error word for non-finite fields.

- Two runs from the same inputs give bit-identical particles (every
  particle's step depends only on the static fields and its own state; the
  sorts are stable); the current agrees to the rounding of the float
  atomics that add the blocks' tiles (their order varies between runs).
- Reading the particles back and loading them into a fresh context resumes
  the run bit-identically (sort cadence aligned).
- The debug launch with one block in flight gives the same particles as the
  normal launch (no interference between concurrent blocks).
- A NaN written into the field buffer raises PIC_DEVERR_NONFINITE."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_17710_amd import workloads as W
from tests import parity_util as U

pytestmark = pytest.mark.gpu

KEYS = ("cell", "offs", "u", "w")


def _wl(geom, seed):
    if geom == "cart3d":
        return W.cart3d(n=16, ppc=4, steps=1, nwaves=8, seed=seed, shuffle=True)
    if geom == "cart2d":
        return W.cart2d(n=32, ppc=8, theta=0.5, steps=1, seed=seed, shuffle=True)
    return W.curvilinear("qsph", 48, 32, 4.0, 0.3, ppc=3, theta=1.0, density_power=0, steps=1,
                         seed=seed, shuffle=True)


def _run(wl, prec, steps, sort_every=3, serial=False):
    import torch

    from paper_2511_17710_amd import picstep as P
    ctx = P.from_workload(wl, prec=prec, sort_every=sort_every)
    if serial:
        ctx.debug_serial(True)
    g = U.oracle_grid(wl)
    dt = O.dt_from_cfl(g, wl.cfl)
    ctx.push_deposit(dt, steps)
    torch.cuda.synchronize()
    parts = [ctx.particles_get(s) for s in range(len(wl.species))]
    return ctx, parts, ctx.current_host().astype(np.float64), dt


def _same_particles(a, b, keys=KEYS):
    for pa, pb in zip(a, b):
        for k in keys:
            np.testing.assert_array_equal(pa[k], pb[k], err_msg=k)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("geom", ["cart3d", "qsph"])
def test_two_runs_are_bit_identical(geom, prec):
    print(f"[robust] determinism {geom} {prec}", flush=True)
    wl = _wl(geom, 91)
    if prec == "f32":
        W.round_to_f32(wl)
    _, a, Ja, _ = _run(wl, prec, 10)
    ctx, b, Jb, _ = _run(wl, prec, 10)
    _same_particles(a, b, KEYS + ("perm", "id", "alive"))
    e = U.rel_l2(Ja, Jb)
    print(f"  current between runs: {e:.2e}", flush=True)
    assert e <= (1e-6 if prec == "f32" else 1e-13)
    assert ctx.device_errors() == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("geom", ["cart3d", "cart2d"])
def test_resume_from_readback_is_bit_identical(geom, prec):
    """12 steps in one context against 6 + 6 with the particles read back
    and loaded into a fresh one in between (sorts every 3 steps, so both
    sort at the same global steps; Cartesian grids: no particle dies)."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[robust] resume {geom} {prec}", flush=True)
    wl = _wl(geom, 92)
    if prec == "f32":
        W.round_to_f32(wl)
    _, whole, Jw, _ = _run(wl, prec, 12)
    _, half, _, dt = _run(wl, prec, 6)
    for sp, p in zip(wl.species, half):
        sp["cell"], sp["offs"], sp["u"], sp["w"] = p["cell"], p["offs"], p["u"], p["w"]
    ctx = P.from_workload(wl, prec=prec, sort_every=3)
    ctx.push_deposit(dt, 6)
    torch.cuda.synchronize()
    resumed = [ctx.particles_get(s) for s in range(len(wl.species))]
    _same_particles(whole, resumed)
    e = U.rel_l2(ctx.current_host().astype(np.float64), Jw)
    print(f"  current of the last step: {e:.2e}", flush=True)
    assert e <= (1e-6 if prec == "f32" else 1e-13)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("geom", ["cart3d", "cart2d", "qsph"])
def test_serial_debug_launch_matches(geom, prec):
    print(f"[robust] one block in flight {geom} {prec}", flush=True)
    wl = _wl(geom, 93)
    if prec == "f32":
        W.round_to_f32(wl)
    _, a, Ja, _ = _run(wl, prec, 4)
    ctx, b, Jb, _ = _run(wl, prec, 4, serial=True)
    _same_particles(a, b, KEYS + ("perm", "alive"))
    e = U.rel_l2(Ja, Jb)
    print(f"  current, normal against serial launch: {e:.2e}", flush=True)
    assert e <= (1e-6 if prec == "f32" else 1e-13)
    assert ctx.device_errors() == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_nonfinite_fields_are_reported(prec):
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[robust] NaN field {prec}", flush=True)
    wl = _wl("cart2d", 94)
    ctx = P.from_workload(wl, prec=prec, sort_every=0)
    g = U.oracle_grid(wl)
    dt = O.dt_from_cfl(g, wl.cfl)
    ctx.push_deposit(dt, 1)
    assert ctx.device_errors() == 0
    ctx.fields()[3, 0, 10, 10] = float("nan")  # B1 at one Yee point
    torch.cuda.synchronize()
    ctx.push_deposit(dt, 1)
    assert ctx.device_errors() & P.PIC_DEVERR_NONFINITE
