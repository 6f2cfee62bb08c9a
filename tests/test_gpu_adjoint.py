"""GPU adjoint of the K-step particle map (Cartesian grids) against the FP64
reference adjoint, against central finite differences of the GPU forward, and
through torch.autograd."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_17710_amd import workloads as W
from tests import parity_util as U

pytestmark = pytest.mark.gpu


def _case(dim, K, seed):
    if dim == 2:
        wl = W.cart2d(n=16, ppc=4, steps=K, seed=seed)
    else:
        wl = W.cart3d(n=8, ppc=2, steps=K, nwaves=8, seed=seed)
    return wl


def _weights(wl, seed):
    rng = np.random.default_rng(seed)
    shp = (3,) + wl.padded_shape()
    lamJ = np.zeros(shp)
    sl = [slice(None)] + [slice(2, 2 + wl.n[d]) if d < wl.dim else slice(None) for d in (2, 1, 0)]
    lamJ[tuple(sl)] = rng.uniform(-1, 1, size=lamJ[tuple(sl)].shape)
    lam_u = [rng.normal(size=(s["cell"].shape[0], 3)) for s in wl.species]
    return lamJ, lam_u


def _gpu_grad(wl, prec, K, m, lamJ, lam_u):
    import torch

    from paper_2511_17710_amd import picstep as P
    ctx = P.from_workload(wl, prec=prec, sort_every=0)
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    ctx.forward_checkpointed(dt, K, m)
    J = ctx.current_host().astype(np.float64)
    L = ctx.layout()
    dtype = torch.float64 if prec == "f64" else torch.float32
    lu = torch.zeros((3, L.capacity), dtype=dtype, device="cuda")
    for s, lam in enumerate(lam_u):
        o = L.species_offset[s]
        lu[:, o:o + lam.shape[0]] = torch.from_numpy(lam.T.copy()).to(dtype=dtype, device="cuda")
    dEB, du0 = ctx.backward(dt, K, m, torch.from_numpy(lamJ).to(dtype=dtype, device="cuda"), lu)
    dEB = dEB.double().cpu().numpy()
    du0 = du0.double().cpu().numpy()
    du = [du0[:, L.species_offset[s]:L.species_offset[s] + lam.shape[0]].T
          for s, lam in enumerate(lam_u)]
    return dEB, du, J, ctx, dt


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim,K,m", [(2, 1, 1), (3, 1, 1), (2, 4, 2), (3, 4, 2)])
def test_adjoint_matches_reference(dim, K, m, prec):
    print(f"[adjoint] dim={dim} K={K} m={m} {prec}", flush=True)
    wl = _case(dim, K, 40 + dim)
    if prec == "f32":
        W.round_to_f32(wl)
    lamJ, lam_u = _weights(wl, 7)
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    ref = O.adjoint(g, dt, K, EB, wl.species, lamJ, lam_u=lam_u)
    dEB, du, J, ctx, _ = _gpu_grad(wl, prec, K, m, lamJ, lam_u)
    _, Jref = O.run(g, dt, K, EB, wl.species)
    eJ = U.rel_l2(J, Jref)
    eE = U.rel_l2(dEB, ref["dEB"])
    eu = U.rel_l2(np.concatenate(du), np.concatenate(ref["du0"]))
    print(f"  J {eJ:.2e} dEB {eE:.2e} du0 {eu:.2e}", flush=True)
    tol = (1e-12 if K == 1 else 1e-10) if prec == "f64" else (1e-5 if K == 1 else 1e-3)
    assert eJ < max(tol, 1e-5 if prec == "f32" else tol)
    assert eE < tol, eE
    assert eu < tol, eu


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_adjoint_with_sorts_inside_the_map(dim, prec):
    """Sorts every 2 steps inside K = 7 steps checkpointed every 3: the
    segments replay the stored permutations and the particle adjoints follow
    every sort back.  lam_u is given in the order at step K (mapped through
    checkpointed_order from per-particle values); du0 comes back in the order
    at step 0 and is compared with the reference adjoint of the unsorted map
    (each particle's gradient does not depend on the order)."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[adjoint] sorts inside dim={dim} {prec}", flush=True)
    K, m, S = 7, 3, 2
    wl = _case(dim, K, 50 + dim)
    if prec == "f32":
        W.round_to_f32(wl)
    lamJ, lam_u = _weights(wl, 11)
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    ref = O.adjoint(g, dt, K, EB, wl.species, lamJ, lam_u=lam_u)
    _, Jref = O.run(g, dt, K, EB, wl.species, sort_every=S)
    ctx = P.from_workload(wl, prec=prec, sort_every=S)
    ctx.forward_checkpointed(dt, K, m)
    J = ctx.current_host().astype(np.float64)
    L = ctx.layout()
    order = ctx.checkpointed_order()
    lu0 = np.zeros((3, L.capacity))
    for s, lam in enumerate(lam_u):
        o = L.species_offset[s]
        lu0[:, o:o + lam.shape[0]] = lam.T
    moved = 0
    for s, lam in enumerate(lam_u):
        o, n = L.species_offset[s], lam.shape[0]
        seg = order[o:o + n]
        assert np.array_equal(np.sort(seg), np.arange(o, o + n))  # a permutation of the species
        moved += int(np.sum(seg != np.arange(o, o + n)))
    assert moved > 0  # the sorts did reorder particles
    dtype = torch.float64 if prec == "f64" else torch.float32
    lu = torch.from_numpy(lu0[:, order].copy()).to(dtype=dtype, device="cuda")
    dEB, du0 = ctx.backward(dt, K, m, torch.from_numpy(lamJ).to(dtype=dtype, device="cuda"), lu)
    dEB = dEB.double().cpu().numpy()
    du0 = du0.double().cpu().numpy()
    du = [du0[:, L.species_offset[s]:L.species_offset[s] + lam.shape[0]].T
          for s, lam in enumerate(lam_u)]
    eJ = U.rel_l2(J, Jref)
    eE = U.rel_l2(dEB, ref["dEB"])
    eu = U.rel_l2(np.concatenate(du), np.concatenate(ref["du0"]))
    print(f"  J {eJ:.2e} dEB {eE:.2e} du0 {eu:.2e}", flush=True)
    tol = 1e-10 if prec == "f64" else 1e-3
    assert eJ < (1e-10 if prec == "f64" else 1e-5)
    assert eE < tol, eE
    assert eu < tol, eu
    # the particles are back at their step-0 state and order
    for s in range(len(wl.species)):
        q = ctx.particles_get(s)
        np.testing.assert_array_equal(q["cell"][:, :dim], wl.species[s]["cell"][:, :dim])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_manual_checkpoints_and_adjoint_steps(prec):
    """pic_checkpoint_save / pic_checkpoint_load / pic_adjoint_step driven by
    the caller reproduce pic_forward_checkpointed + pic_backward."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[adjoint] manual checkpoints {prec}", flush=True)
    K = 4
    wl = _case(3, K, 47)
    if prec == "f32":
        W.round_to_f32(wl)
    lamJ, lam_u = _weights(wl, 12)
    dEB_ref, du_ref, _, _, dt = _gpu_grad(wl, prec, K, 2, lamJ, lam_u)
    ctx = P.from_workload(wl, prec=prec, sort_every=0)
    dtype = torch.float64 if prec == "f64" else torch.float32
    L = ctx.layout()
    slots = [ctx.checkpoint_slot() for _ in range(K)]
    for n in range(K):
        ctx.checkpoint_save(slots[n])
        ctx.push_deposit(dt, 1)
    lu = torch.zeros((3, L.capacity), dtype=dtype, device="cuda")
    for s, lam in enumerate(lam_u):
        o = L.species_offset[s]
        lu[:, o:o + lam.shape[0]] = torch.from_numpy(lam.T.copy()).to(dtype=dtype, device="cuda")
    ld = torch.zeros_like(lu)
    dEB = torch.zeros((6,) + ctx.padded_shape(), dtype=dtype, device="cuda")
    lJ = torch.from_numpy(lamJ).to(dtype=dtype, device="cuda")
    for n in range(K - 1, -1, -1):
        ctx.checkpoint_load(slots[n])
        ctx.adjoint_step(dt, lu, ld, dEB, lamJ=lJ if n == K - 1 else None)
    torch.cuda.synchronize()
    du0 = lu.double().cpu().numpy()
    du = [du0[:, L.species_offset[s]:L.species_offset[s] + lam.shape[0]].T
          for s, lam in enumerate(lam_u)]
    eE = U.rel_l2(dEB.double().cpu().numpy(), dEB_ref)
    eu = U.rel_l2(np.concatenate(du), np.concatenate(du_ref))
    print(f"  dEB {eE:.2e} du0 {eu:.2e}", flush=True)
    assert eu == 0.0 or eu < 1e-14
    assert eE < (1e-13 if prec == "f64" else 1e-6)


def test_checkpoint_interval_does_not_change_gradients():
    """Recomputing from checkpoints reproduces the stored trajectory exactly:
    du0 is bitwise equal for m = K and m = 1; dEB agrees up to the order of
    the atomic sums."""
    print("[adjoint] checkpoint invariance", flush=True)
    K = 6
    wl = _case(3, K, 44)
    lamJ, lam_u = _weights(wl, 8)
    a = _gpu_grad(wl, "f64", K, K, lamJ, lam_u)
    b = _gpu_grad(wl, "f64", K, 1, lamJ, lam_u)
    for x, y in zip(a[1], b[1]):
        np.testing.assert_array_equal(x, y)
    assert U.rel_l2(a[0], b[0]) < 1e-13


def test_adjoint_central_differences_16cube():
    """The 16^3 subcase (65,536 particles, FP64): <grad, v> against central
    differences of the GPU forward map along random directions."""
    import torch
    print("[adjoint] 16^3 finite differences", flush=True)
    K, m = 8, 4
    wl = W.by_name("cart3d_16_fd", K=K, ckpt=m)
    rng = np.random.default_rng(9)
    lamJ = wl.W
    lam_u = [rng.normal(size=(s["cell"].shape[0], 3)) for s in wl.species]
    dEB, du, _, ctx, dt = _gpu_grad(wl, "f64", K, m, lamJ, lam_u)
    g, EB0 = U.oracle_fields(wl, "f64")
    mask = np.zeros_like(EB0, dtype=bool)
    mask[:, 2:18, 2:18, 2:18] = True
    L = ctx.layout()

    def loss(EBx, du_dir, h):
        from paper_2511_17710_amd import picstep as P
        c = P.from_workload(wl, prec="f64", sort_every=0)
        c.fields().copy_(torch.from_numpy(EBx).cuda())
        c.fields_fill_ghosts()
        arr = c.particle_arrays()
        for s, d in enumerate(du_dir):
            o = L.species_offset[s]
            for a in range(3):
                arr["u"][a][o:o + d.shape[0]] += torch.from_numpy(h * d[:, a]).cuda()
        c.push_deposit(dt, K)
        J = c.current_host()
        uu = [c.particles_get(s)["u"] for s in range(len(wl.species))]
        return float(np.sum(lamJ * J) + sum(np.sum(l * x) for l, x in zip(lam_u, uu)))

    # The first-order shape has kinks (relay clamp, half-cell stagger switch):
    # with 65,536 particles x 8 steps a perturbation of 1e-6 carries about one
    # trajectory across a kink (1e-5 relative error); 1e-8 makes that unlikely
    # while FP64 round-off of the difference stays near 3e-7.
    for trial in range(2):
        vE = rng.normal(size=EB0.shape) * mask
        vu = [rng.normal(size=(s["cell"].shape[0], 3)) for s in wl.species]
        h = 1e-8
        fd = (loss(EB0 + h * vE, vu, h) - loss(EB0 - h * vE, vu, -h)) / (2 * h)
        ip = np.sum(dEB * vE) + sum(np.sum(a * b) for a, b in zip(du, vu))
        print(f"  trial {trial}: grad.v {ip:.10e} fd {fd:.10e}", flush=True)
        assert ip == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_autograd_function_matches_direct_backward():
    import torch

    from paper_2511_17710_amd import picstep as P
    from paper_2511_17710_amd.autograd import PushDeposit
    print("[adjoint] autograd", flush=True)
    K, m = 3, 2
    wl = _case(3, K, 45)
    lamJ, lam_u = _weights(wl, 10)
    ref = _gpu_grad(wl, "f64", K, m, lamJ, lam_u)
    ctx = P.from_workload(wl, prec="f64", sort_every=0)
    g, EB = U.oracle_fields(wl, "f64")
    dt = O.dt_from_cfl(g, wl.cfl)
    L = ctx.layout()
    EBt = torch.from_numpy(EB).cuda().requires_grad_(True)
    arr = ctx.particle_arrays()
    u0 = torch.stack([arr["u"][a].clone() for a in range(3)]).requires_grad_(True)
    J, uK = PushDeposit.apply(EBt, u0, ctx, dt, K, m)
    lu = torch.zeros_like(uK)
    for s, lam in enumerate(lam_u):
        o = L.species_offset[s]
        lu[:, o:o + lam.shape[0]] = torch.from_numpy(lam.T.copy()).cuda()
    loss = (J * torch.from_numpy(lamJ).cuda()).sum() + (uK * lu).sum()
    loss.backward()
    np.testing.assert_allclose(EBt.grad.cpu().numpy(), ref[0], rtol=0, atol=1e-12 * np.abs(ref[0]).max())
    du0 = u0.grad.cpu().numpy()
    for s, lam in enumerate(lam_u):
        o = L.species_offset[s]
        np.testing.assert_array_equal(du0[:, o:o + lam.shape[0]].T, ref[1][s])


# --------------------------------------------------------------------------- axisymmetric
def _axi_case(geom, K, seed, sort_every=20):
    """A small hot plasma on a log-r grid reaching r = 3 (cells of ~0.06):
    particles cross cells every few steps, some leave radially, and the
    stretched grid (vartheta = 0.3) is exercised by the quasi-spherical one."""
    vt = 0.3 if geom == "qsph" else 0.0
    wl = W.curvilinear(geom, 32, 16, 3.0, vt, ppc=3, theta=2.0, density_power=0, steps=K,
                       seed=seed)
    wl.sort_every = sort_every
    return wl


def _axi_weights(wl, seed):
    """dL/dJ on every node, ghosts included (curvilinear ghosts keep the
    current of radially exiting particles)."""
    rng = np.random.default_rng(seed)
    lamJ = rng.uniform(-1, 1, size=(3,) + wl.padded_shape())
    lam_u = [rng.normal(size=(s["cell"].shape[0], 3)) for s in wl.species]
    return lamJ, lam_u


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("geom,K,m", [("sph", 1, 1), ("qsph", 1, 1), ("sph", 4, 2), ("qsph", 4, 2)])
def test_adjoint_axisymmetric_matches_reference(geom, K, m, prec):
    print(f"[adjoint] {geom} K={K} m={m} {prec}", flush=True)
    wl = _axi_case(geom, K, 60 + K)
    if prec == "f32":
        W.round_to_f32(wl)
    lamJ, lam_u = _axi_weights(wl, 13)
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    ref = O.adjoint(g, dt, K, EB, wl.species, lamJ, lam_u=lam_u)
    dEB, du, J, ctx, _ = _gpu_grad(wl, prec, K, m, lamJ, lam_u)
    out, Jref = O.run(g, dt, K, EB, wl.species)
    dead = sum(int((s["alive"] == 0).sum()) for s in out)
    eJ = U.rel_l2(J, Jref)
    eE = U.rel_l2(dEB, ref["dEB"])
    eu = U.rel_l2(np.concatenate(du), np.concatenate(ref["du0"]))
    print(f"  J {eJ:.2e} dEB {eE:.2e} du0 {eu:.2e} ({dead} particles left radially)", flush=True)
    tol = (1e-12 if K == 1 else 1e-10) if prec == "f64" else (1e-5 if K == 1 else 1e-3)
    assert eJ < max(tol, 1e-5 if prec == "f32" else tol)
    assert eE < tol, eE
    assert eu < tol, eu


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_axisymmetric_with_sorts(prec):
    """Sorts every 2 steps inside K = 6 steps checkpointed every 4 on the
    stretched quasi-spherical grid: the azimuth adjoints follow the sorts
    back with the momentum and offset adjoints."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[adjoint] qsph sorts inside {prec}", flush=True)
    K, m, S = 6, 4, 2
    wl = _axi_case("qsph", K, 71, sort_every=S)
    if prec == "f32":
        W.round_to_f32(wl)
    lamJ, lam_u = _axi_weights(wl, 14)
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    ref = O.adjoint(g, dt, K, EB, wl.species, lamJ, lam_u=lam_u)
    ctx = P.from_workload(wl, prec=prec, sort_every=S)
    ctx.forward_checkpointed(dt, K, m)
    L = ctx.layout()
    order = ctx.checkpointed_order()
    lu0 = np.zeros((3, L.capacity))
    for s, lam in enumerate(lam_u):
        o = L.species_offset[s]
        lu0[:, o:o + lam.shape[0]] = lam.T
    dtype = torch.float64 if prec == "f64" else torch.float32
    lu = torch.from_numpy(lu0[:, order].copy()).to(dtype=dtype, device="cuda")
    dEB, du0 = ctx.backward(dt, K, m, torch.from_numpy(lamJ).to(dtype=dtype, device="cuda"), lu)
    dEB = dEB.double().cpu().numpy()
    du0 = du0.double().cpu().numpy()
    du = [du0[:, L.species_offset[s]:L.species_offset[s] + lam.shape[0]].T
          for s, lam in enumerate(lam_u)]
    eE = U.rel_l2(dEB, ref["dEB"])
    eu = U.rel_l2(np.concatenate(du), np.concatenate(ref["du0"]))
    print(f"  dEB {eE:.2e} du0 {eu:.2e}", flush=True)
    tol = 1e-10 if prec == "f64" else 1e-3
    assert eE < tol, eE
    assert eu < tol, eu


@pytest.mark.parametrize("geom", ["sph", "qsph"])
def test_adjoint_axisymmetric_central_differences(geom):
    """FP64: <grad, v> against central differences of the GPU forward map
    (fields on every padded node, and the initial momenta)."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[adjoint] {geom} finite differences", flush=True)
    K, m = 5, 2
    wl = _axi_case(geom, K, 80, sort_every=0)
    lamJ, lam_u = _axi_weights(wl, 15)
    rng = np.random.default_rng(16)
    dEB, du, _, ctx, dt = _gpu_grad(wl, "f64", K, m, lamJ, lam_u)
    g, EB0 = U.oracle_fields(wl, "f64")
    L = ctx.layout()

    def loss(EBx, du_dir, h):
        c = P.from_workload(wl, prec="f64", sort_every=0)
        c.fields().copy_(torch.from_numpy(EBx).cuda())
        arr = c.particle_arrays()
        for s, d in enumerate(du_dir):
            o = L.species_offset[s]
            for a in range(3):
                arr["u"][a][o:o + d.shape[0]] += torch.from_numpy(h * d[:, a]).cuda()
        c.push_deposit(dt, K)
        J = c.current_host()
        uu = [c.particles_get(s)["u"] for s in range(len(wl.species))]
        return float(np.sum(lamJ * J) + sum(np.sum(l * x) for l, x in zip(lam_u, uu)))

    for trial in range(2):
        vE = rng.normal(size=EB0.shape) * np.abs(EB0).max()
        vu = [rng.normal(size=(s["cell"].shape[0], 3)) for s in wl.species]
        h = 1e-7
        fd = (loss(EB0 + h * vE, vu, h) - loss(EB0 - h * vE, vu, -h)) / (2 * h)
        ip = np.sum(dEB * vE) + sum(np.sum(a * b) for a, b in zip(du, vu))
        print(f"  trial {trial}: grad.v {ip:.10e} fd {fd:.10e}", flush=True)
        assert ip == pytest.approx(fd, rel=1e-6, abs=1e-9)


_K64_REF = {}


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_K64_24cube(prec):
    """The adjoint workload's recipe (pair plasma in plane waves, loss weights
    on every active edge, sorts every 4 steps inside the map) at 24^3 and
    8 particles per cell per species, over the full K = 64 with checkpoints
    every 8: the whole field gradient and every particle's momentum gradient
    against the reference (which runs on a thread pool, particles split into
    groups).  FP64: 1e-10.  FP32: over 64 steps the FP32 trajectories
    separate from the FP64 ones (the forward current after 64 steps is
    compared too, for scale), and a particle that crosses a cell face at
    another step than its FP64 twin gathers other adjoint currents from then
    on; so the bars are 5e-3 on the relative L2 of both gradients, a median
    per-particle error below 1e-4 and 99 % of the particles within 1e-2."""
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[adjoint] 24^3 K=64 {prec}", flush=True)
    wl = W.cart3d_adjoint(n=24, ppc=8, K=64, ckpt=8)
    if prec == "f32":
        W.round_to_f32(wl)
    g, EB = U.oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    if prec not in _K64_REF:
        _K64_REF.clear()
        _K64_REF[prec] = U.adjoint_by_chunks(g, dt, wl.K, EB, wl.species, wl.W)
    ref = _K64_REF[prec]
    ctx = P.from_workload(wl, prec=prec)
    assert ctx.desc.sort_every == wl.sort_every > 0
    ctx.forward_checkpointed(dt, wl.K, wl.ckpt_every)
    J = ctx.current_host().astype(np.float64)
    dEB, du0 = ctx.backward(dt, wl.K, wl.ckpt_every,
                            torch.from_numpy(wl.W).to(device="cuda", dtype=ctx.dtype))
    torch.cuda.synchronize()
    dEB = dEB.double().cpu().numpy()
    du0 = du0.double().cpu().numpy()
    L = ctx.layout()
    du = np.concatenate([du0[:, L.species_offset[s]:L.species_offset[s] + n].T
                         for s, n in enumerate(r.shape[0] for r in ref["du0"])])
    rdu = np.concatenate(ref["du0"])
    eE = U.rel_l2(dEB, ref["dEB"])
    eu = U.rel_l2(du, rdu)
    pp = np.linalg.norm(du - rdu, axis=1) / np.maximum(np.linalg.norm(rdu, axis=1), 1e-30)
    _, Jref = O.run(g, dt, wl.K, EB, wl.species, sort_every=wl.sort_every)
    eJ = U.rel_l2(J, Jref)
    print(f"  forward J {eJ:.2e}; dEB {eE:.2e} du0 {eu:.2e}; per particle du0: median "
          f"{np.median(pp):.2e}, 99th percentile {np.quantile(pp, 0.99):.2e}", flush=True)
    if prec == "f64":
        assert eE < 1e-10 and eu < 1e-10 and eJ < 1e-10, (eE, eu, eJ)
    else:
        assert eE < 5e-3 and eu < 5e-3, (eE, eu)
        assert np.median(pp) < 1e-4 and np.mean(pp < 1e-2) >= 0.99
