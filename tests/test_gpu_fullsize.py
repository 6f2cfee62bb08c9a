"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times (all species in one launch per step, 1024-particle chunks,
LDS current tiles, the workload's sort cadence).

At these sizes the FP64 reference cannot run the whole workload in seconds,
so every check uses outputs it can compute piecewise:
- sampled particles: each particle's state after the run depends only on its
  own initial state and the static fields, so the reference runs the sampled
  particles alone and every one must match;
- a sub-box of the current: a current value at a node only receives deposits
  from particles whose cell at the start of the last step lies within a few
  cells of it, so the reference runs exactly those particles and the box
  must match element by element;
- charge continuity of the GPU's own step over the whole grid (a property
  that holds at any size);
- the adjoint: the gradient with respect to a particle's initial momentum
  depends only on that particle's trajectory, so sampled particles are
  compared with the reference adjoint of those particles alone.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_17710_amd import workloads as W
from tests import checks
from tests import parity_util as U

pytestmark = pytest.mark.gpu

def _workload(name):
    print(f"[fullsize] {name}", flush=True)
    return U.cached_workload(name)


def _subset(species, idx):
    return {k: (v[idx] if isinstance(v, np.ndarray) else v) for k, v in species.items()}


def _gpu(wl, prec, calls):
    """Runs the library for the given numbers of steps per call; returns the
    per-call sort permutations, the final particles and the final current."""
    import torch

    from paper_2511_17710_amd import picstep as P
    ctx = P.from_workload(wl, prec=prec)
    g, _ = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    perms = []
    for k in calls:
        ctx.push_deposit(dt, k)
        torch.cuda.synchronize()
        perms.append([ctx.particles_get(s)["perm"] for s in range(len(wl.species))])
    out = [ctx.particles_get(s) for s in range(len(wl.species))]
    J = ctx.current_host().astype(np.float64)
    del ctx
    torch.cuda.empty_cache()
    return perms, out, J, dt


def _original_index(perms, s, i):
    """Index in the loaded order of the particle now at position i."""
    j = i
    for p in reversed(perms):
        j = p[s][j]
    return j


def _check_samples(wl, prec, perms, gpu, dt, steps, nsample, rng):
    g, EB = U.oracle_fields(wl, prec)
    worst_u, mism = 0.0, 0
    for s, q in enumerate(gpu):
        n = q["cell"].shape[0]
        pick = np.sort(rng.choice(n, size=min(nsample, n), replace=False))
        orig = _original_index(perms, s, pick)
        np.testing.assert_array_equal(q["id"][pick], orig)  # ids carried through every sort
        sub = _subset(wl.species[s], orig)
        ref, _ = O.run(g, dt, steps, EB, [sub], sort_every=0)
        r = ref[0]
        np.testing.assert_array_equal(q["alive"][pick], r["alive"])
        live = r["alive"] == 1
        du = np.linalg.norm(q["u"][pick] - r["u"], axis=1)
        rel = du / np.maximum(np.linalg.norm(r["u"], axis=1), 1e-3)
        same = np.all(q["cell"][pick] == r["cell"], axis=1)
        if prec == "f64":
            assert same[live].all(), f"{(~same[live]).sum()} cell mismatches"
            doff = np.abs(q["offs"][pick] - r["offs"])[live]
            assert doff.max(initial=0) <= 1e-11, doff.max()
        else:
            mism += int((~same & live).sum())
        worst_u = max(worst_u, float(rel[live].max(initial=0)))
        if r["phi"] is not None:
            dphi = np.abs((q["phi"][pick] - r["phi"] + np.pi) % (2 * np.pi) - np.pi)[live]
            assert dphi.max(initial=0) <= (1e-11 if prec == "f64" else 1e-4)
    print(f"  samples: u rel err {worst_u:.2e}, cell mismatches {mism}", flush=True)
    if prec == "f64":
        assert worst_u < 1e-11
    else:
        assert worst_u < 1e-4
        assert mism <= max(3, 1e-4 * nsample * len(gpu))


def _check_box(wl, prec, perms, gpu, Jg, dt, steps, lo, size, compare_j=True):
    """Current on the nodes [lo, lo + size) of every active dimension against
    the reference run of every particle that can reach them."""
    g, EB = U.oracle_fields(wl, prec)
    subs, sels = [], []
    for s, q in enumerate(gpu):
        sel = np.ones(q["cell"].shape[0], dtype=bool)
        for d in range(wl.dim):
            c = q["cell_prev"][:, d].astype(np.int64)
            if wl.geom == "cart":  # periodic: distance along the ring
                sel &= np.mod(c - (lo[d] - 3), wl.n[d]) <= size[d] + 5
            else:
                sel &= (c >= lo[d] - 3) & (c <= lo[d] + size[d] + 2)
        idx = np.nonzero(sel)[0]
        sels.append(idx)
        subs.append(_subset(wl.species[s], _original_index(perms, s, idx)))
    _, Jref = O.run(g, dt, steps, EB, subs, sort_every=0)
    nodes = []
    for d in (2, 1, 0):
        nodes.append(slice(lo[d] + 2, lo[d] + 2 + size[d]) if d < wl.dim else slice(None))
    a, b = Jg[(slice(None),) + tuple(nodes)], Jref[(slice(None),) + tuple(nodes)]
    e = U.rel_l2(a, b)
    # charge continuity on the box nodes from the GPU's own positions of the
    # same particles (extended precision)
    pc = np.concatenate([q["cell_prev"][i] for q, i in zip(gpu, sels)])
    po = np.concatenate([q["offs_prev"][i] for q, i in zip(gpu, sels)])
    nc = np.concatenate([q["cell"][i] for q, i in zip(gpu, sels)])
    no = np.concatenate([q["offs"][i] for q, i in zip(gpu, sels)])
    qw = np.concatenate([sp["q"] * q["w"][i] for sp, q, i in zip(wl.species, gpu, sels)])
    c = checks.continuity_residual_box(Jg, wl.n, wl.dim, wl.geom == "cart", dt, (pc, po),
                                       (nc, no), qw, tuple(nodes))
    print(f"  box {lo} x {size}: {len(qw)} particles, J rel L2 {e:.2e}, continuity {c:.2e}",
          flush=True)
    assert np.abs(b).max() > 0
    if compare_j:
        assert e < (1e-11 if prec == "f64" else 1e-4), e
    assert c < (1e-12 if prec == "f64" else 1e-6), c


def _check_continuity(wl, prec, gpu, Jg, dt):
    """Whole-grid continuity with FP64 charge sums (FP32 builds and the 3D
    box, whose steps move particles a fair fraction of a cell); the FP64
    axisymmetric steps move particles ~1e-4 cell and rely on the
    extended-precision box checks."""
    pc = np.concatenate([q["cell_prev"] for q in gpu])
    po = np.concatenate([q["offs_prev"] for q in gpu])
    nc = np.concatenate([q["cell"] for q in gpu])
    no = np.concatenate([q["offs"] for q in gpu])
    qw = np.concatenate([sp["q"] * q["w"] for sp, q in zip(wl.species, gpu)])
    c = checks.continuity_residual_fast(Jg, wl.n, wl.dim, wl.geom == "cart", dt, (pc, po),
                                        (nc, no), qw)
    print(f"  continuity residual {c:.2e}", flush=True)
    assert c < (1e-12 if prec == "f64" else 1e-6), c


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cart3d_128_full(prec):
    """67,108,864 particles, 6 steps with the workload's cadence of 5: a sort
    before the first and before the sixth step."""
    print(f"[fullsize] cart3d_128 {prec}", flush=True)
    wl = _workload("cart3d_128")
    if prec == "f32":
        W.round_to_f32(wl)
    assert wl.sort_every == 5
    perms, gpu, Jg, dt = _gpu(wl, prec, (1, 5))
    rng = np.random.default_rng(11)
    _check_samples(wl, prec, perms, gpu, dt, 6, 3000, rng)
    _check_box(wl, prec, perms, gpu, Jg, dt, 6, (40, 70, 100), (10, 10, 10))
    _check_box(wl, prec, perms, gpu, Jg, dt, 6, (0, 0, 120), (6, 6, 8))  # periodic seams
    _check_continuity(wl, prec, gpu, Jg, dt)


def _check_all(wl, prec, gpu, Jg, dt):
    """The whole one-step run (sort at step 0, then the step) through the
    reference: permutations bit-exact, every particle, the whole current."""
    g, EB = U.oracle_fields(wl, prec)
    # momentum scale |k E_p|; in the cells the step takes in FP64 (within 2
    # cells of the axis and of r_min, where E can nearly vanish at the
    # particle while its stencil nodes do not) the interpolated |E| stencil
    # magnitude instead, when larger
    ks_pt = U.kick_scale(wl, g, EB, dt)
    ks_st = U.kick_scale(wl, g, EB, dt, stencil=True)
    ks = []
    for s, sp in enumerate(wl.species):
        c = sp["cell"]
        near = (c[:, 0] < 2) | (c[:, 1] < 2) | (c[:, 1] >= wl.n[1] - 2)
        ks.append(np.where(near, np.maximum(ks_pt[s], ks_st[s]), ks_pt[s]))
        print(f"  species {s}: {int(near.sum())} of {near.size} particles in the FP64 cells "
              f"take the stencil scale", flush=True)
    ref, Jref = O.run(g, dt, 1, EB, wl.species, sort_every=wl.sort_every)
    tol = U.TOL[prec]
    for s, (r, q) in enumerate(zip(ref, gpu)):
        perm = r["perm"]
        np.testing.assert_array_equal(q["perm"], perm)
        np.testing.assert_array_equal(q["alive"], r["alive"])
        err_u = U.momentum_error(r, q, wl.species[s]["u"][perm], ks[s][perm])
        same = np.all(q["cell"] == r["cell"], axis=1)
        if prec == "f64":
            assert same.all(), f"{(~same).sum()} cell mismatches"
        else:
            bad = ~same & ~U.near_face(r["offs"][:, :wl.dim], 1e-5)
            assert not bad.any(), f"{bad.sum()} cell mismatches away from faces"
        doff = np.abs(q["offs"] - r["offs"])[same]
        print(f"  species {s}: u err {err_u:.2e}, offsets {doff.max(initial=0):.2e}", flush=True)
        assert err_u <= tol["u"], err_u
        assert doff.max(initial=0) <= tol["offs"], doff.max()
    e = U.rel_l2(Jg, Jref)
    # in-plane current of the GPU's own (stored) trajectory, deposited in FP64
    pc = np.concatenate([q["cell_prev"] for q in gpu])
    po = np.concatenate([q["offs_prev"] for q in gpu])
    nc = np.concatenate([q["cell"] for q in gpu])
    no = np.concatenate([q["offs"] for q in gpu])
    qw = np.concatenate([sp["q"] * q["w"] for sp, q in zip(wl.species, gpu)])
    Jz = checks.zigzag_current(wl.n, wl.dim, wl.geom == "cart", dt, qw, (pc, po), (nc, no))
    k = 2 if wl.dim == 2 else 3
    e_own = U.rel_l2(Jg[:k], Jz[:k])
    # out-of-plane current (2D) against the reference, on the scale of the
    # whole current: for a cold start it is second order (the azimuthal
    # displacement of an initially resting particle is a small difference of
    # Cartesian displacements) and carries no significant digits of its own
    e_out = (float(np.linalg.norm(Jg[2] - Jref[2]) / np.linalg.norm(Jref))
             if wl.dim == 2 else 0.0)
    cold = all(not np.any(sp["u"]) for sp in wl.species)
    print(f"  whole current: J rel L2 {e:.2e}; in-plane vs own trajectory {e_own:.2e}; "
          f"out-of-plane {e_out:.2e}{' (cold start)' if cold else ''}", flush=True)
    assert e_own <= tol["J"], e_own
    assert e_out <= tol["J"], e_out
    if prec == "f32" and cold:
        # From rest, the first step moves outer particles ~1e-9 cell; the
        # stored FP32-build offsets resolve 2^-32 cell, so the stored
        # trajectory (checked above) differs from the FP64 one by up to half
        # a quantum, and co-located pairs moving apart by less than that do
        # not separate at all.  The in-plane current follows the stored
        # trajectory exactly; against FP64 it is bounded by that rounding.
        assert e <= 1e-4, e
    else:
        assert e <= tol["J"], e


@pytest.mark.parametrize("name,prec,whole", [
    ("qsph_1024x512", "f64", True), ("qsph_1024x512", "f32", True),
    ("sph_1024x512", "f32", True), ("qsph_2048x1024", "f32", True),
    ("qsph_2048x1024", "f64", False)])
def test_curvilinear_full(name, prec, whole):
    """The axisymmetric workloads at full size: sort, then one step.  Where
    the reference can run the whole workload in well under a minute it does,
    and everything is compared; the FP64 run of the 67M-particle grid is
    checked by samples and boxes."""
    print(f"[fullsize] {name} {prec}", flush=True)
    wl = _workload(name)
    if prec == "f32":
        W.round_to_f32(wl)
    perms, gpu, Jg, dt = _gpu(wl, prec, (1,))
    if whole:
        _check_all(wl, prec, gpu, Jg, dt)
    else:
        rng = np.random.default_rng(12)
        _check_samples(wl, prec, perms, gpu, dt, 1, 3000, rng)
    n1, n2 = wl.n[0], wl.n[1]
    # boxes: the current against the reference, and charge continuity of the
    # GPU's own step in extended precision (FP32: the current of the outer
    # corner, where cold particles move ~1e-9 cell per step, is only as
    # accurate as the 2^-32 offsets; the whole-current bar covers it)
    jbox = prec == "f64"
    _check_box(wl, prec, perms, gpu, Jg, dt, 1, (n1 // 3, n2 // 3, 0), (24, 24, 1), jbox)
    _check_box(wl, prec, perms, gpu, Jg, dt, 1, (0, 0, 0), (8, 8, 1), jbox)  # r_min, the axis
    _check_box(wl, prec, perms, gpu, Jg, dt, 1, (n1 - 8, n2 - 8, 0), (8, 8, 1), jbox)
    if prec == "f32":
        _check_continuity(wl, prec, gpu, Jg, dt)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_cart3d_64_full(prec):
    """The adjoint workload at full size (4,194,304 particles, K = 64,
    checkpoints every 8, the workload's sort cadence inside the map, as the
    benchmark runs it): sampled gradients with respect to the initial
    momenta (returned in the loaded order)."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[fullsize] adjoint cart3d_64 {prec}", flush=True)
    wl = W.by_name("cart3d_64_adj")
    if prec == "f32":
        W.round_to_f32(wl)
    K, m = wl.K, wl.ckpt_every
    ctx = P.from_workload(wl, prec=prec)
    assert wl.sort_every > 0
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    lamJ = torch.from_numpy(wl.W).to(device="cuda", dtype=ctx.dtype)
    ctx.forward_checkpointed(dt, K, m)
    _, du0 = ctx.backward(dt, K, m, lamJ)
    torch.cuda.synchronize()
    du0 = du0.double().cpu().numpy()
    L = ctx.layout()
    rng = np.random.default_rng(13)
    errs = []
    for s in range(len(wl.species)):
        n = wl.species[s]["cell"].shape[0]
        pick = np.sort(rng.choice(n, size=200, replace=False))
        sub = _subset(wl.species[s], pick)
        ref = O.adjoint(g, dt, K, EB, [sub], wl.W)
        gp = du0[:, L.species_offset[s] + pick].T
        rp = ref["du0"][0]
        errs.append(np.linalg.norm(gp - rp, axis=1) / np.maximum(np.linalg.norm(rp, axis=1), 1e-30))
    e = np.concatenate(errs)
    print(f"  du0 rel err: max {e.max():.2e} median {np.median(e):.2e}", flush=True)
    assert np.isfinite(e).all()
    if prec == "f64":
        assert e.max() < 1e-9
    else:
        # a trajectory that crosses a face at a different step than the FP64
        # one (offsets within FP32 rounding of the face) gathers different
        # adjoint currents; such particles must stay rare
        assert np.median(e) < 1e-4
        assert np.mean(e < 1e-2) >= 0.99


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_cart3d_64_subbox_fields(prec):
    """The full 64^3 adjoint workload over K = 8 (checkpoints every 4, sorts
    inside the map): the field gradient on a 12^3 block of nodes against the
    reference adjoint of the particles that start within 6 cells of the
    block.  In 8 steps a particle moves at most 8 c dt < 2.1 cells and its
    interpolation and deposit stencils reach 2 cells, so no other particle
    touches the block.  Bars: 1e-10 (FP64), 1e-3 (FP32)."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[fullsize] adjoint cart3d_64 K=8 sub-box {prec}", flush=True)
    K, m = 8, 4
    wl = _workload("cart3d_64_adj")
    if prec == "f32":
        W.round_to_f32(wl)
    ctx = P.from_workload(wl, prec=prec)
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    assert K * dt < 2.1
    ctx.forward_checkpointed(dt, K, m)
    dEB, _ = ctx.backward(dt, K, m, torch.from_numpy(wl.W).to(device="cuda", dtype=ctx.dtype))
    torch.cuda.synchronize()
    dEB = dEB.double().cpu().numpy()
    lo, size, margin = 26, 12, 6
    near = []
    for sp in wl.species:
        c = sp["cell"]
        near.append(U.subset_species(sp, np.nonzero(np.all((c >= lo - margin) & (c < lo + size + margin),
                                                           axis=1))[0]))
    ref = U.adjoint_by_chunks(g, dt, K, EB, near, wl.W)
    blk = (slice(None),) + (slice(W.NG + lo, W.NG + lo + size),) * 3
    e = U.rel_l2(dEB[blk], ref["dEB"][blk])
    print(f"  {sum(s['cell'].shape[0] for s in near)} particles near the block; dEB rel {e:.2e}",
          flush=True)
    tol = 1e-10 if prec == "f64" else 1e-3
    assert e < tol
