"""GPU field solver (Faraday, Ampere with the axis rules, current filter) and
the whole loop of Sec. 2.3 against the FP64 reference, from the GPU's own
stored fields (so both sides start from the same values).

Bars: FP64 build 1e-12 (one solver call) and 1e-10 (the loop over several
steps, particles included); FP32 build 1e-6 relative L2 for one solver call
(the kernels combine in FP64 and round once), the loop reported with 1e-4
(trajectories of the FP32 particle step separate at the 1e-7 level and the
fields follow them)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_17710_amd import workloads as W
from tests import checks
from tests import parity_util as U

pytestmark = pytest.mark.gpu

NG = 2


def _wl(geom):
    if geom == "cart2d":
        return W.cart2d(n=24, ppc=4, theta=0.5, steps=1, seed=71, shuffle=True)
    if geom == "cart3d":
        return W.cart3d(n=8, ppc=2, steps=1, nwaves=8, seed=72, shuffle=True)
    if geom == "sph":
        return W.curvilinear("sph", 32, 16, 4.0, 0.0, ppc=3, theta=1.0, density_power=0, steps=1,
                             seed=73, shuffle=True)
    return W.curvilinear("qsph", 32, 16, 4.0, 0.3, ppc=3, theta=1.0, density_power=0, steps=1,
                         seed=74, shuffle=True)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("geom", ["cart2d", "cart3d", "sph", "qsph"])
def test_solver_pieces_match_reference(geom, prec):
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[fields] solver pieces {geom} {prec}", flush=True)
    wl = _wl(geom)
    if prec == "f32":
        W.round_to_f32(wl)
    ctx = P.from_workload(wl, prec=prec, sort_every=0)
    g = U.oracle_grid(wl)
    rng = np.random.default_rng(5)
    tol = 1e-12 if prec == "f64" else 1e-6
    EB = ctx.fields_host().astype(np.float64)
    # Faraday
    f = 0.5 * O.dt_from_cfl(g, wl.cfl)
    ctx.fields_advance_b(f)
    got = ctx.fields_host().astype(np.float64)
    ref = O.faraday(g, EB, f)
    eB = _rel(got[3:], ref[3:])
    assert np.array_equal(got[:3], EB[:3])
    # Ampere with a random current (ghosts included: curvilinear ghost current
    # is kept, periodic ghosts are zero after a step)
    J = rng.normal(size=(3,) + ctx.padded_shape()) * 0.05
    if wl.geom == "cart":
        Jz = np.zeros_like(J)
        sl = [slice(None)] + [slice(NG, NG + wl.n[d]) if d < wl.dim else slice(None)
                              for d in (2, 1, 0)]
        Jz[tuple(sl)] = J[tuple(sl)]
        J = Jz
    ctx.current().copy_(torch.from_numpy(J).to(dtype=ctx.dtype, device="cuda"))
    J = ctx.current_host().astype(np.float64)
    dt = O.dt_from_cfl(g, wl.cfl)
    ctx.fields_advance_e(dt, 4 * np.pi)
    got2 = ctx.fields_host().astype(np.float64)
    ref2 = O.ampere(g, got, J, dt, 4 * np.pi)
    eE = _rel(got2[:3], ref2[:3])
    # filter passes
    ctx.current_filter(3)
    gotJ = ctx.current_host().astype(np.float64)
    refJ = O.filter_current(g, J, 3)
    eJ = _rel(gotJ, refJ)
    print(f"  faraday {eB:.2e} ampere {eE:.2e} filter {eJ:.2e}", flush=True)
    assert eB <= tol and eE <= tol and eJ <= tol, (eB, eE, eJ)
    if wl.geom != "cart":  # the axis rules
        for c in (2, 4):
            assert not np.any(got2[c, :, [NG, NG + wl.n[1]], :])


def _reference_loop(wl, prec, K, passes, coupling):
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    species = wl.species
    J = None
    for n in range(K):
        EB = O.faraday(g, EB, 0.5 * dt)
        species, J = O.run(g, dt, 1, EB, species, sort_every=wl.sort_every, step0=n)
        if passes:
            J = O.filter_current(g, J, passes)
        EB = O.faraday(g, EB, 0.5 * dt)
        EB = O.ampere(g, EB, J, dt, coupling)
    return species, EB, J, dt


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("geom", ["cart2d", "qsph"])
def test_full_loop_matches_reference(geom, prec):
    """Five steps of the whole loop (Faraday half, particle step with the
    sort cadence, two filter passes, Faraday half, Ampere) on both sides."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[fields] full loop {geom} {prec}", flush=True)
    K, passes, coupling = 5, 2, 4 * np.pi * 0.05
    wl = _wl(geom)
    wl.sort_every = 2
    if prec == "f32":
        W.round_to_f32(wl)
    ref, EBr, Jr, dt = _reference_loop(wl, prec, K, passes, coupling)
    ctx = P.from_workload(wl, prec=prec)
    ctx.step_full(dt, K, passes, coupling)
    torch.cuda.synchronize()
    EBg = ctx.fields_host().astype(np.float64)
    Jg = ctx.current_host().astype(np.float64)
    eF = _rel(EBg, EBr)
    eJ = _rel(Jg, Jr)
    worst_u, mism = 0.0, 0
    for s, r in enumerate(ref):
        q = ctx.particles_get(s)
        np.testing.assert_array_equal(q["perm"], r["perm"])
        same = np.all(q["cell"] == r["cell"], axis=1)
        mism += int((~same).sum())
        du = np.linalg.norm(q["u"] - r["u"], axis=1) / np.maximum(np.linalg.norm(r["u"], axis=1), 1e-3)
        worst_u = max(worst_u, float(du.max()))
    print(f"  fields {eF:.2e} current {eJ:.2e} u {worst_u:.2e} cell mismatches {mism}", flush=True)
    if prec == "f64":
        assert eF < 1e-10 and eJ < 1e-10 and worst_u < 1e-10 and mism == 0
    else:
        assert eF < 1e-4 and eJ < 1e-4 and worst_u < 1e-4


def test_gauss_law_over_the_loop_periodic():
    """FP64, 2D periodic box: div E - coupling rho stays the same at every
    node over the whole loop (the deposit conserves charge exactly and the
    discrete divergence of a discrete curl vanishes); filtering is off, as
    the filter does not preserve the local charge balance."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print("[fields] Gauss's law over 20 steps", flush=True)
    wl = W.cart2d(n=32, ppc=8, theta=0.5, steps=1, seed=77)
    coupling = 4 * np.pi * 0.02
    ctx = P.from_workload(wl, prec="f64")
    g = U.oracle_grid(wl)
    dt = O.dt_from_cfl(g, wl.cfl)
    n = wl.n

    def gauss():
        E = ctx.fields_host()[:3]
        div = checks.divergence(E, n, 2, True).astype(np.float64)
        parts = [ctx.particles_get(s) for s in range(len(wl.species))]
        rho = sum(checks.rho_nodes(n, 2, True, p["cell"], p["offs"],
                                   sp["q"] * p["w"]).astype(np.float64)
                  for sp, p in zip(wl.species, parts))
        # scale: one species' charge (the e-/e+ pairs start co-located, so
        # the total charge density starts at zero)
        rho0 = checks.rho_nodes(n, 2, True, parts[0]["cell"], parts[0]["offs"],
                                wl.species[0]["q"] * parts[0]["w"]).astype(np.float64)
        sl = (0, slice(NG, NG + n[1]), slice(NG, NG + n[0]))
        return div[sl] - coupling * rho[sl], np.abs(coupling * rho0[sl]).max()

    g0, scale = gauss()
    ctx.step_full(dt, 20, 0, coupling)
    torch.cuda.synchronize()
    g1, _ = gauss()
    err = np.abs(g1 - g0).max() / scale
    print(f"  change of div E - coupling rho: {err:.2e} of max |coupling rho|", flush=True)
    assert err < 1e-12
