"""The allocation-free sort (pic_sort_static) against pic_sort, through the C
ABI: two contexts hold the same unsorted particles, one sorts with each entry
point, and every particle array and the permutation must agree bit for bit.
Two calls in a row, the second with fewer particles (the static array keeps
the first call's contents), then a species above the static limit must be
refused before any device work."""
import numpy as np
import pytest

from paper_2511_17710_amd import workloads as W

pytestmark = pytest.mark.gpu


def _shuffled(n, ppc, seed):
    wl = W.cart2d(n=n, ppc=ppc, steps=1, seed=seed, shuffle=True)
    return W.round_to_f32(wl)


def _ctx(wl, prec, cap):
    from paper_2511_17710_amd import picstep as P
    ctx = P.Context(wl.geom, wl.dim, wl.n, wl.lo, wl.hi, periodic=wl.periodic, rho0=wl.rho0,
                    prec=prec, sort_every=0, max_particles=len(wl.species) * cap)
    for s in wl.species:
        ctx.species_add(s["q"], s["m"], cap)
    ctx.bind()
    ctx.fields_set(wl.fields_tetrad, "tetrad", 0)
    return ctx


def _load(ctx, wl):
    for i, s in enumerate(wl.species):
        ctx.particles_load(i, s["cell"], s["offs"], s["u"], s["w"], s.get("phi"))


def _same(a, b, nspec):
    for s in range(nspec):
        qa, qb = a.particles_get(s), b.particles_get(s)
        for k in ("perm", "id", "cell", "offs", "u", "w", "alive"):
            np.testing.assert_array_equal(qa[k], qb[k], err_msg=f"species {s} {k}")
        assert not np.array_equal(qa["perm"], np.arange(qa["perm"].shape[0]))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_sort_static_matches_sort(prec):
    import torch

    from paper_2511_17710_amd import picstep as P
    print(f"[no_alloc] sort_static vs sort, {prec}", flush=True)
    big = _shuffled(256, 32, 5)      # 2 x 2,097,152 particles
    small = _shuffled(96, 20, 6)     # 2 x 184,320 particles (other grid size)
    cap = big.species[0]["cell"].shape[0]
    ref, sta = _ctx(big, prec, cap), _ctx(big, prec, cap)
    _load(ref, big)
    _load(sta, big)
    ref.sort()
    sta.sort_static()
    torch.cuda.synchronize()
    _same(ref, sta, len(big.species))
    # second call on a smaller input: fresh contexts on another grid
    ref2, sta2 = _ctx(small, prec, cap), _ctx(small, prec, cap)
    _load(ref2, small)
    _load(sta2, small)
    ref2.sort()
    sta2.sort_static()
    torch.cuda.synchronize()
    _same(ref2, sta2, len(small.species))
    # and the first contexts again, after a step (a pending reorder is applied first)
    dt = ref.timestep_from_cfl(big.cfl)
    for c in (ref, sta):
        c.push_deposit(dt, 2)
    ref.sort()
    sta.sort_static()
    torch.cuda.synchronize()
    _same(ref, sta, len(big.species))
    del ref, sta, ref2, sta2
    torch.cuda.empty_cache()


def test_sort_static_refuses_above_limit():
    import torch

    from paper_2511_17710_amd import picstep as P
    print("[no_alloc] limit", flush=True)
    wl = _shuffled(512, 17, 7)  # 4,456,448 per species > 2^22
    n = wl.species[0]["cell"].shape[0]
    assert n > (1 << 22)
    ctx = _ctx(wl, "f32", n)
    _load(ctx, wl)
    with pytest.raises(P.PicError) as e:
        ctx.sort_static()
    assert e.value.status == P.PIC_E_CAPACITY
    assert "at most 4194304" in str(e.value)
    ctx.sort()  # the context is unaffected
    torch.cuda.synchronize()
    del ctx
    torch.cuda.empty_cache()
