"""Per-step parity along the full benchmark runs (GPU vs the FP64 reference).

Each workload runs on the GPU for its whole length (the 128^3 box 100 steps,
the axisymmetric grids 200), in the benchmark's launch configuration and sort
cadence.  At steps {0, mid, last} the GPU's own particle state is read back
and handed to the reference, and one step is taken on both sides from that
common state.  This isolates the error of one step from the divergence of
trajectories that accumulates over many steps (which is not asserted).

Per checkpoint:
- momenta of sampled particles (or of every particle, where the reference
  runs the whole grid in seconds): max |u_gpu - u_ref| / max(|u_old|,
  |u_ref|, |k E_p|); next to the polar axis, where the interpolated E nearly
  cancels while the stored node values do not, the scale also takes |k| times
  the interpolated |E| of the stencil (the count of such particles is printed);
- cell indices (FP64 bit-exact; FP32 exact away from faces) and offsets;
- the sort permutation, when the step began with a sort: bit-exact against
  the reference's stable sort of the GPU's own keys;
- the current on boxes of nodes (every particle that can reach them run by
  the reference), or on the whole grid: relative L2 error;
- charge continuity of the GPU's own step on the whole grid.

Bars (FP32 / FP64): momenta 1e-5 / 1e-12, current 1e-5 / 1e-12, continuity
1e-6 / 1e-12.  The one exception is the first step of the cold 1024x512
workload in FP32, whose current error is printed, not asserted: from rest the
outer particles move about 1e-9 cell in that step, below the 2^-32 cell
resolution of the stored offsets (mid and last steps are asserted).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_17710_amd import workloads as W
from tests import checks
from tests import parity_util as U

pytestmark = pytest.mark.gpu

KEYS = ("cell", "offs", "u", "w", "phi", "alive", "id")


def _get(ctx, s, prev=False):
    q = ctx.particles_get(s)
    keep = KEYS + (("cell_prev", "offs_prev", "perm") if prev else ())
    return {k: q[k] for k in keep}


def _aligned(before, after):
    """The state before the step in the order after it (matched by id)."""
    n = before["id"].shape[0]
    inv = np.empty(n, dtype=np.int64)
    inv[before["id"]] = np.arange(n)
    idx = inv[after["id"]]
    return {k: (v[idx] if isinstance(v, np.ndarray) else v) for k, v in before.items()}, idx


def _species(sp, st, sel=None):
    out = {"q": sp["q"], "m": sp["m"]}
    for k in ("cell", "offs", "u", "w", "phi", "alive"):
        v = st[k]
        out[k] = None if v is None else (v if sel is None else v[sel])
    return out


def _kick(wl, g, EB, dt, st, axis_cells):
    """|k E_p| and, for particles within axis_cells of theta = 0 or pi, the
    stencil scale |k| |sqrt(h) sum w |E^i||."""
    F = O.interp(g, EB, st["cell"], st["offs"])
    E, _ = O.to_cart(g, st["cell"], st["offs"], st["phi"], F)
    k = abs(st["q"] * dt / (2 * st["m"] * wl.rho0))
    ks = k * np.linalg.norm(E, axis=1)
    nstencil = 0
    if wl.geom != "cart":
        j = st["cell"][:, 1]
        near = (j < axis_cells) | (j >= wl.n[1] - axis_cells)
        if near.any():
            Fa = O.interp(g, np.abs(EB), st["cell"][near], st["offs"][near])
            Ea, _ = O.to_cart(g, st["cell"][near], st["offs"][near], st["phi"][near], Fa)
            ks[near] = np.maximum(ks[near], k * np.linalg.norm(Ea, axis=1))
            nstencil = int(near.sum())
    return ks, nstencil


def _compare_particles(wl, prec, g, EB, dt, sp, bef, aft, sel, tag, r=None):
    """One reference step of the selected particles from the GPU's state
    before the step (r: that step, when already run); momenta, cells and
    offsets against the GPU's state after it."""
    tol = U.TOL[prec]
    sub = _species(sp, bef, sel)
    if r is None:
        r = O.run(g, dt, 1, EB, [sub], sort_every=0)[0][0]
    q = {k: aft[k][sel] for k in ("cell", "offs", "u", "phi", "alive")
         if aft.get(k) is not None}
    np.testing.assert_array_equal(q["alive"], r["alive"])
    live = (sub["alive"] == 1)
    ks, nst = _kick(wl, g, EB, dt, sub, 2)
    du = np.linalg.norm(q["u"] - r["u"], axis=1)
    den = np.maximum.reduce([np.linalg.norm(sub["u"], axis=1), np.linalg.norm(r["u"], axis=1),
                             ks, np.full(du.shape, 1e-30)])
    err_u = float((du / den)[live].max(initial=0.0))
    same = np.all(q["cell"] == r["cell"], axis=1)
    alive_now = r["alive"] == 1
    if prec == "f64":
        bad = int((~same & alive_now).sum())
    else:
        bad = int((~same & alive_now & ~U.near_face(r["offs"][:, :wl.dim], 1e-5)).sum())
    near = int((~same & alive_now).sum())
    doff = np.abs(q["offs"] - r["offs"])[same & alive_now]
    e_off = float(doff.max(initial=0.0))
    e_phi = 0.0
    if r["phi"] is not None:
        dphi = np.abs((q["phi"] - r["phi"] + np.pi) % (2 * np.pi) - np.pi)[alive_now]
        e_phi = float(dphi.max(initial=0.0))
    print(f"  {tag}: {int(live.sum())} particles, u err {err_u:.2e} "
          f"({nst} on the stencil scale), cells differing {near} (away from faces {bad}), "
          f"offsets {e_off:.2e}, phi {e_phi:.2e}", flush=True)
    assert err_u <= tol["u"], err_u
    assert bad == 0, bad
    assert e_off <= tol["offs"], e_off
    assert e_phi <= (1e-11 if prec == "f64" else 2e-5), e_phi


def _box_sel(wl, st, lo, size):
    sel = np.ones(st["cell"].shape[0], dtype=bool)
    for d in range(wl.dim):
        c = st["cell"][:, d].astype(np.int64)
        if wl.geom == "cart":
            sel &= np.mod(c - (lo[d] - 3), wl.n[d]) <= size[d] + 5
        else:
            sel &= (c >= lo[d] - 3) & (c <= lo[d] + size[d] + 2)
    return np.nonzero(sel)[0]


def _box_nodes(wl, lo, size):
    nodes = []
    for d in (2, 1, 0):
        nodes.append(slice(lo[d] + 2, lo[d] + 2 + size[d]) if d < wl.dim else slice(None))
    return (slice(None),) + tuple(nodes)


def _run_case(name, prec, checkpoints, boxes, whole, nsample, cold_first=False):
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[perstep] {name} {prec}: generating", flush=True)
    wl = U.cached_workload(name)
    if prec == "f32":
        W.round_to_f32(wl)
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    ctx = P.from_workload(wl, prec=prec)
    se = wl.sort_every
    nspec = len(wl.species)
    tol = U.TOL[prec]
    rng = np.random.default_rng(17)
    done = 0
    for step in checkpoints:
        if step > done:
            ctx.push_deposit(dt, step - done)
        torch.cuda.synchronize()
        before = [_get(ctx, s) for s in range(nspec)]
        ctx.push_deposit(dt, 1)
        torch.cuda.synchronize()
        done = step + 1
        after = [_get(ctx, s, prev=True) for s in range(nspec)]
        Jg = ctx.current_host().astype(np.float64)
        sorted_here = se > 0 and step % se == 0
        print(f"[perstep] {name} {prec} step {step}{' (sort)' if sorted_here else ''}",
              flush=True)
        al = []
        for s in range(nspec):
            b, a = before[s], after[s]
            n = b["id"].shape[0]
            assert np.array_equal(np.sort(a["id"]), np.arange(n)), "ids not a permutation"
            ba, idx = _aligned(b, a)
            al.append(ba)
            # the GPU's prev positions are its own state before the step
            np.testing.assert_array_equal(a["cell_prev"][:, :wl.dim], ba["cell"][:, :wl.dim])
            np.testing.assert_array_equal(a["offs_prev"][:, :wl.dim], ba["offs"][:, :wl.dim])
            if sorted_here:
                keys = O.sort_keys(g, b["cell"], b["alive"])
                perm = O.sort_perm(keys)
                np.testing.assert_array_equal(a["perm"], perm)
                np.testing.assert_array_equal(idx, perm)
        if whole:
            subs = [_species(wl.species[s], al[s]) for s in range(nspec)]
            ref, Jref = O.run(g, dt, 1, EB, subs, sort_every=0)
            for s in range(nspec):
                allp = np.arange(al[s]["id"].shape[0])
                _compare_particles(wl, prec, g, EB, dt, wl.species[s], al[s], after[s], allp,
                                   f"species {s} (all)", r=ref[s])
            e = U.rel_l2(Jg, Jref)
            print(f"  whole current: J rel L2 {e:.2e}", flush=True)
            if cold_first and prec == "f32" and step == 0:
                assert e <= 1e-4, e  # reported; see the module docstring
            else:
                assert e <= tol["J"], e
        else:
            for s in range(nspec):
                n = al[s]["id"].shape[0]
                pick = np.sort(rng.choice(n, size=min(nsample, n), replace=False))
                _compare_particles(wl, prec, g, EB, dt, wl.species[s], al[s], after[s], pick,
                                   f"species {s} (sample)")
            for lo, size in boxes:
                sels = [_box_sel(wl, al[s], lo, size) for s in range(nspec)]
                subs = [_species(wl.species[s], al[s], sels[s]) for s in range(nspec)]
                _, Jref = O.run(g, dt, 1, EB, subs, sort_every=0)
                nodes = _box_nodes(wl, lo, size)
                a_, b_ = Jg[nodes], Jref[nodes]
                assert np.abs(b_).max() > 0
                e = U.rel_l2(a_, b_)
                print(f"  box {lo} x {size}: {sum(len(x) for x in sels)} particles, "
                      f"J rel L2 {e:.2e}", flush=True)
                if cold_first and prec == "f32" and step == 0:
                    assert e <= 1e-4, e
                else:
                    assert e <= tol["J"], e
        # charge continuity of the GPU's own step: FP64 charge sums where
        # particles move a fair fraction of a cell (the 3D box; the hot
        # 2048x1024 plasma in FP32), the telescoped charge change where the
        # whole grid is checked, boxes in extended precision otherwise
        pc = np.concatenate([a["cell_prev"] for a in after])
        po = np.concatenate([a["offs_prev"] for a in after])
        nc = np.concatenate([a["cell"] for a in after])
        no = np.concatenate([a["offs"] for a in after])
        qw = np.concatenate([sp["q"] * a["w"] for sp, a in zip(wl.species, after)])
        cart = wl.geom == "cart"
        if whole:
            c = checks.continuity_residual_telescoped(Jg, wl.n, wl.dim, cart, dt, (pc, po),
                                                      (nc, no), qw)
            print(f"  continuity residual (telescoped) {c:.2e}", flush=True)
            assert c <= tol["cont"], c
        elif cart or prec == "f32":
            c = checks.continuity_residual_fast(Jg, wl.n, wl.dim, cart, dt, (pc, po), (nc, no),
                                                qw)
            print(f"  continuity residual {c:.2e}", flush=True)
            assert c <= tol["cont"], c
        else:
            # particles dead before the step (outside the radial range) did not move
            was_alive = (pc[:, 0] >= 0) & (pc[:, 0] < wl.n[0])
            for lo, size in boxes:
                sel = _box_sel(wl, {"cell": pc}, lo, size)
                sel = sel[was_alive[sel]]
                c = checks.continuity_residual_box(Jg, wl.n, wl.dim, cart, dt,
                                                   (pc[sel], po[sel]), (nc[sel], no[sel]),
                                                   qw[sel], _box_nodes(wl, lo, size)[1:])
                print(f"  continuity residual on box {lo} {c:.2e}", flush=True)
                assert c <= tol["cont"], c
        del before, after, al, pc, po, nc, no, qw
    del ctx
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_perstep_cart3d_128(prec):
    """128^3 box, 67,108,864 particles, 100 steps with a sort every 5."""
    _run_case("cart3d_128", prec, (0, 50, 99),
              boxes=[((40, 70, 100), (10, 10, 10)), ((0, 0, 120), (6, 6, 8))],
              whole=False, nsample=3000)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_perstep_qsph_1024x512(prec):
    """Cold pair plasma on the 1024x512 log-r grid, 200 steps, whole grid."""
    _run_case("qsph_1024x512", prec, (0, 100, 199), boxes=[], whole=True, nsample=0,
              cold_first=True)


def test_perstep_sph_1024x512():
    """The uniform-r spherical metric at the same size, FP32, whole grid."""
    _run_case("sph_1024x512", "f32", (0, 100, 199), boxes=[], whole=True, nsample=0,
              cold_first=True)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_perstep_qsph_2048x1024(prec):
    """Hot plasma on the stretched 2048x1024 grid (67,108,864 particles),
    200 steps with a sort every 20: samples and boxes at the inner radius and
    axis, mid-grid, and the outer radius at theta = pi."""
    _run_case("qsph_2048x1024", prec, (0, 100, 199),
              boxes=[((0, 0, 0), (8, 8, 1)), ((680, 340, 0), (24, 24, 1)),
                     ((2040, 1016, 0), (8, 8, 1))],
              whole=False, nsample=3000)
