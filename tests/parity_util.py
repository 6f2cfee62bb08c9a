"""Runs one workload through the FP64 reference and through the HIP library
from the same seeded inputs, and measures their agreement."""
import copy

import numpy as np

from oracle import oracle as O
from paper_2511_17710_amd import workloads as W
from tests import checks

TOL = {  # GPU vs FP64 reference, one step from a common state
    "f32": dict(u=1e-5, J=1e-5, cont=1e-6, offs=1e-5),
    "f64": dict(u=1e-12, J=1e-12, cont=1e-12, offs=1e-12),
}


def oracle_grid(wl):
    return O.make_grid(wl.geom, wl.dim, wl.n, wl.lo, wl.hi, r0=wl.r0, vartheta=wl.vartheta,
                       periodic=wl.periodic, rho0=wl.rho0)


def oracle_fields(wl, prec):
    g = oracle_grid(wl)
    EB = O.fields_from_tetrad(g, wl.fields_tetrad, wl.fields_includes_ghosts)
    if prec == "f32":
        EB = EB.astype(np.float32).astype(np.float64)
    return g, EB


def kick_scale(wl, g, EB, dt, stencil=False):
    """|k E_p| per particle of every species at the initial state (reference).

    stencil=True interpolates |E| instead: |k| times the norm of
    sqrt(h_ii) sum_nodes w |E^i|, the scale of the rounding error of the
    interpolation sum (where E nearly vanishes at the particle, e.g. next to
    the polar axis, the stored node values set the error, not their sum)."""
    out = []
    for s in wl.species:
        F = O.interp(g, np.abs(EB) if stencil else EB, s["cell"], s["offs"])
        E, _ = O.to_cart(g, s["cell"], s["offs"], s.get("phi"), F)
        k = s["q"] * dt / (2 * s["m"] * wl.rho0)
        out.append(np.abs(k) * np.linalg.norm(E, axis=1))
    return out


def run_both(wl, prec, steps, sort_every=None, print_case=None):
    """Returns (reference species, reference J, gpu species, gpu J, dt)."""
    import torch

    from paper_2511_17710_amd import picstep as P
    if print_case:
        print(print_case, flush=True)
    if prec == "f32":
        W.round_to_f32(wl)
    se = wl.sort_every if sort_every is None else sort_every
    g, EB = oracle_fields(wl, prec)
    dt = O.dt_from_cfl(g, wl.cfl)
    ref, Jref = O.run(g, dt, steps, EB, wl.species, sort_every=se)
    ctx = P.from_workload(wl, prec=prec, sort_every=se)
    assert abs(ctx.timestep_from_cfl(wl.cfl) - dt) <= 1e-14 * dt
    ctx.push_deposit(dt, steps)
    torch.cuda.synchronize()
    gpu = [ctx.particles_get(s) for s in range(len(wl.species))]
    Jg = ctx.current_host().astype(np.float64)
    return ref, Jref, gpu, Jg, dt, ctx


def momentum_error(ref_sp, gpu_sp, u_old, kscale):
    du = np.linalg.norm(gpu_sp["u"] - ref_sp["u"], axis=1)
    den = np.maximum.reduce([np.linalg.norm(u_old, axis=1), np.linalg.norm(ref_sp["u"], axis=1),
                             kscale, np.full(du.shape, 1e-30)])
    return float(np.max(du / den)) if du.size else 0.0


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def continuity_of(wl, J, species, dt):
    pc = np.concatenate([s["cell_prev"] for s in species])
    po = np.concatenate([s["offs_prev"] for s in species])
    nc = np.concatenate([s["cell"] for s in species])
    no = np.concatenate([s["offs"] for s in species])
    qw = np.concatenate([sp["q"] * s["w"] for sp, s in zip(wl.species, species)])
    return checks.continuity_residual(J, wl.n, wl.dim, wl.geom == "cart", dt, (pc, po), (nc, no), qw)


def near_face(offs, tol):
    return np.any((offs < tol) | (offs > 1 - tol), axis=1)


_WL_CACHE = {}


def cached_workload(name):
    """A deep copy of a full-size workload, generated once while consecutive
    tests ask for the same one (one kept at a time: they are large)."""
    if name not in _WL_CACHE:
        _WL_CACHE.clear()
        _WL_CACHE[name] = W.by_name(name)
    return copy.deepcopy(_WL_CACHE[name])


def adjoint_by_chunks(g, dt, K, EB, species, lamJ, nthreads=None):
    """The reference adjoint of the particle map over disjoint groups of
    particles on a thread pool (the library call releases the interpreter
    lock).  The loss is linear in the final current and the particles do not
    act on each other within the map, so the field gradient is the sum of
    the groups' and each particle's gradient is its group's."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    nthreads = nthreads or min(16, os.cpu_count() or 1)
    jobs = []
    for s, sp in enumerate(species):
        n = sp["cell"].shape[0]
        for idx in np.array_split(np.arange(n), nthreads):
            if idx.size:
                jobs.append((s, idx))

    def one(job):
        s, idx = job
        return O.adjoint(g, dt, K, EB, [subset_species(species[s], idx)], lamJ)

    with ThreadPoolExecutor(nthreads) as ex:
        res = list(ex.map(one, jobs))
    dEB = sum(r["dEB"] for r in res)
    du0 = [np.zeros((sp["cell"].shape[0], 3)) for sp in species]
    for (s, idx), r in zip(jobs, res):
        du0[s][idx] = r["du0"][0]
    return dict(dEB=dEB, du0=du0)


def subset_species(sp, idx):
    """The particles idx of one species (per-particle arrays indexed, the
    species' constants kept)."""
    out = {}
    for k, v in sp.items():
        if isinstance(v, np.ndarray) and v.ndim >= 1 and v.shape[0] == sp["cell"].shape[0]:
            out[k] = v[idx]
        else:
            out[k] = v
    return out
